"""Pins of the oracle's direct sampler (oracle/sampling.py, Sec. 2 chain
rule) against exact enumeration: the histogram of its samples over every
configuration of a small lattice follows P(s) = exp(2 log psi(s)) from the
full forward pass (chi-square test on bins of expected count >= 10), the
log psi it returns is the forward pass's, and the draw rule's edge cases
hold.  A sampler that read the wrong class, conditioned on the wrong sites
or dropped the factor 1/2 fails one of these."""
from dataclasses import replace
import itertools

import numpy as np
import pytest
from scipy.stats import chi2

from oracle import network as net
from oracle import sampling
from workloads import CONFIGS, make_params


def _all_states(N):
    return np.array(list(itertools.product([1, -1], repeat=N)),
                    dtype=np.int8)


def _chi2_pvalue(samples, states, probs, min_expected=10.0):
    """Chi-square p-value of the sample histogram against probs, with
    states pooled (in order of probability) into bins of expected count at
    least min_expected."""
    S = samples.shape[0]
    idx = {s.tobytes(): k for k, s in enumerate(states)}
    counts = np.zeros(len(states))
    for s in samples:
        counts[idx[s.tobytes()]] += 1
    order = np.argsort(probs)
    obs, exp_ = [], []
    o = e = 0.0
    for k in order:
        o += counts[k]
        e += probs[k] * S
        if e >= min_expected:
            obs.append(o)
            exp_.append(e)
            o = e = 0.0
    obs[-1] += o
    exp_[-1] += e
    obs, exp_ = np.array(obs), np.array(exp_)
    stat = ((obs - exp_) ** 2 / exp_).sum()
    return chi2.sf(stat, len(obs) - 1), len(obs)


@pytest.mark.parametrize("L,S", [(3, 40000), (4, 20000)])
def test_histogram_matches_exact_enumeration(L, S):
    mc = replace(CONFIGS["small"], L=L, periodic=(L == 4), batch=S)
    theta = make_params(mc, std=0.4)          # a distribution far from flat
    P = net.unpack(mc, theta)
    states = _all_states(mc.N)
    probs = np.exp(2.0 * net.logpsi_fn(mc, P, chunk=8192)(states))
    assert abs(probs.sum() - 1.0) < 1e-12
    u = np.random.default_rng(90 + L).random((S, mc.N))
    s, lp, _ = sampling.sample(mc, theta, u)
    pval, nbins = _chi2_pvalue(s, states, probs)
    assert nbins > 20
    assert pval > 1e-3, (pval, nbins)


def test_logpsi_is_the_forward_pass_and_draw_rule():
    mc = CONFIGS["small"]
    theta = make_params(mc)
    P = net.unpack(mc, theta)
    u = np.random.default_rng(5).random((64, mc.N))
    s, lp, p_up = sampling.sample(mc, theta, u)
    ref = net.forward(mc, P, s)
    assert np.allclose(lp, ref["logpsi"], rtol=0, atol=1e-12)
    # the compared probabilities are the forward pass's conditionals of +1
    assert np.allclose(p_up, np.exp(ref["lp"][:, :, 0]), rtol=0, atol=1e-14)
    assert np.array_equal(s == 1, u < p_up)
    # u = 0 always draws +1; u just below 1 draws -1 (0 < p < 1)
    s0, _, _ = sampling.sample(mc, theta, np.zeros((2, mc.N)))
    assert (s0 == 1).all()
    s1, _, _ = sampling.sample(mc, theta,
                               np.full((2, mc.N), 1.0 - 2.0 ** -53))
    assert (s1 == -1).all()
