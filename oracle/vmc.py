"""One variational Monte Carlo step, FP64 (paper Sec. 2, eqs. 1-3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a real, positive psi the energy E = <psi|H|psi> / <psi|psi> =
E_s~psi^2 [E_loc(s)] (eq. 1) has the gradient

    dE/dtheta = 2 E_s~psi^2 [ (E_loc(s) - E) d log psi(s) / d theta ],

(eq. 3 for a zero phase).  Over a batch of B direct samples the estimate is
the batch mean with E replaced by the batch mean of E_loc:
weights w_i = 2 (E_loc(s_i) - mean) / B on the per-sample gradients of
log psi (straight-through across the quantizer, eqs. 7-8).  The step is
then theta <- theta - lr * gradient.

``energy_gradient_exact`` is the same expression with the expectation over
every configuration weighted by P(s) = psi(s)^2 (small lattices only).
"""
import itertools

import numpy as np

from . import eloc as oeloc
from . import grad as ograd
from . import sampling


def sample_weights(E):
    E = np.asarray(E, dtype=np.float64)
    return 2.0 * (E - E.mean()) / E.size


def energy_gradient_samples(cfg, theta, spins):
    """(gradient estimate [P], E_loc [B]) over the batch of samples."""
    E = oeloc.eloc_network_naive(cfg, theta, spins)
    return ograd.grad_logpsi(cfg, theta, spins, weights=sample_weights(E)), E


def energy_gradient_exact(cfg, theta):
    """(dE/dtheta [P], E) with the expectation over all 2^N configurations
    weighted by P(s) = exp(2 log psi(s))."""
    N = cfg.N
    states = np.array(list(itertools.product([1, -1], repeat=N)),
                      dtype=np.int8)
    lp = ograd.logpsi(cfg, theta, states)
    p = np.exp(2.0 * lp)
    E_loc = oeloc.eloc_network_naive(cfg, theta, states)
    E = float((p * E_loc).sum())
    w = 2.0 * p * (E_loc - E)
    return ograd.grad_logpsi(cfg, theta, states, weights=w), E


def vmc_step_sgd(cfg, theta, uniforms, lr):
    """One step: samples from the uniforms, local energies, the gradient
    estimate, theta - lr * gradient.  Returns (new theta, spins, E_loc)."""
    spins, _, _ = sampling.sample(cfg, theta, uniforms)
    g, E = energy_gradient_samples(cfg, theta, spins)
    return np.asarray(theta, dtype=np.float64) - lr * g, spins, E
