"""Pins of the oracle's VMC energy gradient (oracle/vmc.py, eq. 3).

With one codeword per quantizer head the quantized vector is a constant,
so the straight-through gradient is the true derivative, and the exact
expectation 2 E_psi^2[(E_loc - E) d log psi] must equal central finite
differences of the exact energy <psi|H|psi>/<psi|psi>, with H from the
independent Pauli-matrix construction (oracle/ed.py).  A dropped factor 2,
a missing mean subtraction or a wrong sign fails this.  The batch form is
the exact form with the sample mean in place of the expectation."""
from dataclasses import replace

import numpy as np

from oracle import ed
from oracle import grad as ograd
from oracle import vmc
from oracle.eloc import eloc_network_naive
from workloads import CONFIGS, make_params, param_layout


def _exact_energy(cfg, theta, H):
    import itertools
    states = np.array(list(itertools.product([1, -1], repeat=cfg.N)),
                      dtype=np.int8)
    psi = np.exp(ograd.logpsi(cfg, theta, states))
    idx = ed.index_of_config(states)
    v = np.zeros(2 ** cfg.N)
    v[idx] = psi
    return float(v @ (H @ v) / (v @ v))


def test_exact_gradient_equals_finite_differences_of_the_energy():
    mc = replace(CONFIGS["small"], L=3, periodic=False, d_model=8,
                 n_heads=2, d_ff=16, codebook_size=1, n_layers=1)
    theta = make_params(mc, std=0.3)
    H = ed.hamiltonian(mc.L, mc.periodic, mc.J, mc.marshall)
    g, E = vmc.energy_gradient_exact(mc, theta)
    assert abs(E - _exact_energy(mc, theta, H)) < 1e-12 * abs(E)
    lay = {name: off for name, _, _, off, _ in param_layout(mc)}
    rng = np.random.default_rng(3)
    picks = [lay["pos_emb"] + 5, lay["l0.W1"] + 7, lay["l0.b2"] + 1,
             lay["W_head"] + 3, lay["lnf_g"] + 2, lay["tok_emb"] + 9,
             lay["l0.codebook"] + 1]
    h = 1e-6
    for k in picks:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (_exact_energy(mc, tp, H) - _exact_energy(mc, tm, H)) / (2 * h)
        assert abs(g[k] - fd) < 1e-6 * max(1.0, abs(fd)), (k, g[k], fd)


def test_batch_estimate_is_the_weighted_sum_with_sample_mean():
    mc = replace(CONFIGS["small"], batch=6)
    theta = make_params(mc)
    spins = np.random.default_rng(4).choice([1, -1], size=(6, mc.N)) \
        .astype(np.int8)
    g, E = vmc.energy_gradient_samples(mc, theta, spins)
    assert np.allclose(E, eloc_network_naive(mc, theta, spins), rtol=0,
                       atol=1e-12)
    per = ograd.grad_logpsi(mc, theta, spins)
    ref = (2.0 / 6) * ((E - E.mean())[:, None] * per).sum(axis=0)
    assert np.allclose(g, ref, rtol=1e-12, atol=1e-12)
