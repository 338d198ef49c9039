"""Pins of the oracle's bidirectional encoder with mean pooling used as
log psi (Sec. 3.1: the encoder network pools the hidden states of its last
layer and maps them linearly to a scalar), against what the definition and
the mathematics fix independently of the oracle's code:

* all weights zero except the head bias b: log psi = b for every
  configuration, so every ratio is 1 and E_loc = diag + h n_neighbours
  (h = -J/2) in closed form;
* with zero position embeddings the network is symmetric under any
  permutation of the tokens (attention over all positions, per-location
  operations, a mean), which a causal mask or a position-dependent pooling
  would break;
* the attention is bidirectional: changing the last token changes the
  first position's attention output;
* the deduplicated local energy (every row attends again, the mean pooled
  over the changed rows) equals the plain re-evaluation of eq. (2);
* the straight-through gradient matches central differences.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import eloc as oeloc
from oracle import grad as og
from oracle import lattice
from oracle import network as net
from workloads import CONFIGS, make_params, make_spins
from workloads.layout import param_layout, param_count

ENC = replace(CONFIGS["small"], name="small_enc", encoder=True, batch=6)
ENC4 = replace(ENC, name="small_enc_g4", group=4)


def _slice(mc, name):
    return [(o, n) for nm, shape, kind, o, n in param_layout(mc)
            if nm == name][0]


@pytest.mark.parametrize("mc", [ENC, ENC4], ids=["K1", "K4"])
def test_zero_weights_closed_form(mc):
    theta = np.zeros(param_count(mc))
    off, _ = _slice(mc, "b_head")
    theta[off] = 0.37
    s = make_spins(mc)
    P = net.unpack(mc, theta)
    assert np.allclose(net.forward(mc, P, s)["logpsi"], 0.37, rtol=0,
                       atol=1e-15)
    E = oeloc.eloc_network_naive(mc, theta, s)
    bl = lattice.bonds(mc.L, mc.periodic)
    diag = lattice.diagonal(s, bl, mc.J)
    h = lattice.offdiag_element(mc.J, mc.marshall)
    nnb = np.array([len(lattice.neighbours(s[b], bl)) for b in range(len(s))])
    assert np.allclose(E, diag + h * nnb, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mc", [ENC, ENC4], ids=["K1", "K4"])
def test_permutation_symmetry_without_positions(mc):
    theta = make_params(mc, std=0.3)
    off, n = _slice(mc, "pos_emb")
    theta[off:off + n] = 0.0
    P = net.unpack(mc, theta)
    s = make_spins(mc)
    rng = np.random.default_rng(8)
    K, T = mc.group, mc.N // mc.group
    perm = rng.permutation(T)
    sites = (perm[:, None] * K + np.arange(K)[None, :]).reshape(-1)
    lp = net.forward(mc, P, s)["logpsi"]
    lq = net.forward(mc, P, s[:, sites])["logpsi"]
    assert np.allclose(lp, lq, rtol=0, atol=1e-12)
    # the decoder with the same weights is not symmetric (it is causal)
    dec = replace(mc, encoder=False)
    th_d = make_params(dec, std=0.3)
    od, nd = _slice(dec, "pos_emb")
    th_d[od:od + nd] = 0.0
    Pd = net.unpack(dec, th_d)
    assert not np.allclose(net.forward(dec, Pd, s)["logpsi"],
                           net.forward(dec, Pd, s[:, sites])["logpsi"])


def test_attention_is_bidirectional():
    mc = ENC
    P = net.unpack(mc, make_params(mc))
    s = make_spins(mc)[:1]
    t = s.copy()
    t[0, -1] = -t[0, -1]
    a0 = net.forward(mc, P, s, keep=True)["caches"][0]["a"][0, 0]
    a1 = net.forward(mc, P, t, keep=True)["caches"][0]["a"][0, 0]
    assert np.abs(a0 - a1).max() > 1e-6


@pytest.mark.parametrize("mc", [ENC, ENC4], ids=["K1", "K4"])
def test_dedup_equals_plain(mc):
    theta = make_params(mc)
    s = make_spins(mc)[:3]
    E_d, info = oeloc.eloc_dedup(mc, theta, s, return_info=True)
    E_n = oeloc.eloc_network_naive(mc, theta, s)
    assert np.allclose(E_d, E_n, rtol=1e-12, atol=0)
    # every row of every neighbour went through attention again
    assert all(r == mc.n_layers * (mc.N // mc.group) for r in info["att_rows"])


def test_central_differences():
    mc = replace(ENC, d_model=8, n_heads=2, d_ff=16, codebook_size=6,
                 vq_heads=2, n_layers=2)
    th = make_params(mc)
    s = make_spins(mc)[:1]
    g = og.grad_logpsi(mc, th, s)[0]
    fr = og.frozen_state(mc, th, s)
    rng = np.random.default_rng(9)
    eps = 1e-6
    for _ in range(5):
        v = rng.standard_normal(th.size)
        v /= np.linalg.norm(v)
        fp = og.surrogate_logpsi(mc, th + eps * v, s, fr)[0]
        fm = og.surrogate_logpsi(mc, th - eps * v, s, fr)[0]
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g @ v) <= 1e-7 * (1 + abs(fd)), (fd, g @ v)
    lp = og.logpsi(mc, th, s)
    assert np.allclose(lp, net.forward(mc, net.unpack(mc, th), s)["logpsi"],
                       rtol=0, atol=1e-12)
