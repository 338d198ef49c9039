"""Pins of the oracle with tokens of K > 1 spins (Sec. 3.1: tokens are
groups of K particles with a vocabulary of d^K values; the paper's
experiments use groups of 4), against what the definition and the
mathematics fix independently of the oracle's code:

* the token of a group, worked by hand for a fixed spin row;
* all weights zero except the head bias b: every conditional is
  softmax(b), so log psi(s) = 1/2 sum_i log softmax(b)[t_i] in closed form;
* the distribution sums to one over all 2^16 states of the 4x4 lattice
  (autoregressive normalisation, Sec. 2), for K = 2 and K = 4;
* direct samples follow that exact distribution (chi-square) and their
  log psi is the forward pass's;
* the deduplicated local energy equals the plain re-evaluation of eq. (2)
  (every neighbour's network evaluated from scratch), exchanges within one
  token and across two included;
* the straight-through gradient matches central differences of the
  surrogate (the embedding and head tensors, whose shapes change with K,
  included).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import eloc as oeloc
from oracle import grad as og
from oracle import lattice
from oracle import network as net
from oracle import sampling
from workloads import CONFIGS, make_params, make_spins
from workloads.layout import param_layout, param_count

from test_oracle_sampling import _all_states, _chi2_pvalue

G4 = replace(CONFIGS["small"], name="small_g4", group=4, batch=8)
G2 = replace(CONFIGS["small"], name="small_g2", group=2, batch=8)


def test_token_of_a_group_by_hand():
    s = np.array([[1, -1, -1, 1, -1, -1, -1, -1]], dtype=np.int8)
    t, u = net.tokens(s, 4)
    # bits (site k of the group, 1 for spin -1): 0110 -> 2 + 4 = 6; 1111 -> 15
    assert t.tolist() == [[6, 15]]
    assert u.tolist() == [[16, 6]]          # BOS = 2^4, then the shift
    t1, u1 = net.tokens(s, 1)
    assert t1.tolist() == [[0, 1, 1, 0, 1, 1, 1, 1]]
    assert u1.tolist() == [[2, 0, 1, 1, 0, 1, 1, 1]]


@pytest.mark.parametrize("mc", [G2, G4], ids=["K2", "K4"])
def test_layout_sizes(mc):
    V, T, d = 1 << mc.group, mc.N // mc.group, mc.d_model
    lay = {name: (shape, n) for name, shape, kind, off, n in param_layout(mc)}
    assert lay["tok_emb"][0] == (V + 1, d)
    assert lay["pos_emb"][0] == (T, d)
    assert lay["W_head"][0] == (d, V) and lay["b_head"][0] == (V,)
    assert param_count(mc) == net.n_params(mc)


@pytest.mark.parametrize("mc", [G2, G4], ids=["K2", "K4"])
def test_zero_weights_closed_form(mc):
    theta = np.zeros(param_count(mc))
    b = np.random.default_rng(3).standard_normal(1 << mc.group)
    off = [o for name, shape, kind, o, n in param_layout(mc)
           if name == "b_head"][0]
    theta[off:off + b.size] = b
    logsm = b - np.log(np.exp(b).sum())
    s = make_spins(mc)
    t, _ = net.tokens(s, mc.group)
    expect = 0.5 * logsm[t].sum(axis=1)
    got = net.forward(mc, net.unpack(mc, theta), s)["logpsi"]
    assert np.allclose(got, expect, rtol=0, atol=1e-13)


@pytest.mark.parametrize("mc", [G2, G4], ids=["K2", "K4"])
def test_normalised_over_all_states(mc):
    theta = make_params(mc, std=0.4)
    P = net.unpack(mc, theta)
    probs = np.exp(2.0 * net.logpsi_fn(mc, P, chunk=8192)(_all_states(mc.N)))
    assert abs(probs.sum() - 1.0) < 1e-12


def test_sampler_histogram_and_logpsi_k4():
    mc = replace(G4, batch=1 << 17)
    theta = make_params(mc, std=0.4)
    P = net.unpack(mc, theta)
    states = _all_states(mc.N)
    probs = np.exp(2.0 * net.logpsi_fn(mc, P, chunk=8192)(states))
    u = np.random.default_rng(91).random((mc.batch, mc.N))
    s, lp, pr = sampling.sample(mc, theta, u)
    assert pr.shape == (mc.batch, mc.T, 16)
    pval, nbins = _chi2_pvalue(s, states, probs)
    assert nbins > 100
    assert pval > 1e-3, (pval, nbins)
    ref = net.forward(mc, P, s[:256])["logpsi"]
    assert np.allclose(lp[:256], ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mc", [G2, G4], ids=["K2", "K4"])
def test_dedup_equals_plain(mc):
    theta = make_params(mc)
    s = make_spins(mc)[:3]
    E_d, info = oeloc.eloc_dedup(mc, theta, s, return_info=True)
    E_n = oeloc.eloc_network_naive(mc, theta, s)
    assert np.allclose(E_d, E_n, rtol=1e-12, atol=0)
    # both kinds of exchange occur: sites in one token and in two
    bl = lattice.bonds(mc.L, mc.periodic)
    kinds = {p1 // mc.group == p2 // mc.group
             for b in range(3) for _, p1, p2 in lattice.neighbours(s[b], bl)}
    assert kinds == {True, False}


def test_central_differences_k4():
    mc = replace(G4, d_model=8, n_heads=2, d_ff=16, codebook_size=6,
                 vq_heads=2, n_layers=2)
    th = make_params(mc)
    s = make_spins(mc)[:1]
    g = og.grad_logpsi(mc, th, s)[0]
    fr = og.frozen_state(mc, th, s)
    rng = np.random.default_rng(6)
    eps = 1e-6
    lay = {name: (off, n) for name, shape, kind, off, n in param_layout(mc)}
    dirs = []
    for name in ("tok_emb", "W_head", "b_head"):
        off, n = lay[name]
        v = np.zeros(th.size)
        v[off:off + n] = rng.standard_normal(n)
        dirs.append(v / np.linalg.norm(v))
    for _ in range(3):
        v = rng.standard_normal(th.size)
        dirs.append(v / np.linalg.norm(v))
    for v in dirs:
        fp = og.surrogate_logpsi(mc, th + eps * v, s, fr)[0]
        fm = og.surrogate_logpsi(mc, th - eps * v, s, fr)[0]
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g @ v) <= 1e-7 * (1 + abs(fd)), (fd, g @ v)
