"""Oracle pins for the VQ transformer (CPU only).

* Autoregressive normalisation: sum over all 2^N configurations of
  psi(s)^2 = P(s) equals 1 (chain rule, Sec. 2).  Catches a missing input
  shift, a leaky causal mask, a wrong log-softmax or a wrong factor 1/2.
* Causal-prefix invariance (Sec. 2 discussion of autoregressive reuse).
* Each operation against an independent library routine: LayerNorm,
  causal scaled-dot-product attention and exact GELU from torch; nearest
  codeword (eqs. 4-6) against torch.cdist brute force, with ties to the
  lowest index and exact codewords.
* Permuting attention heads (with the matching columns/rows) leaves psi
  unchanged.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import network as net
from workloads import CONFIGS, make_params, make_spins, param_count, with_batch
from workloads.layout import param_layout


def all_configs(N):
    idx = np.arange(2 ** N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N)) & 1
    return np.where(bits == 1, -1, 1).astype(np.int8)


@pytest.mark.parametrize("name", ["small", "medium", "large", "grad"])
def test_param_count_matches_layout(name):
    cfg = CONFIGS[name]
    assert net.n_params(cfg) == param_count(cfg)
    theta = np.arange(param_count(cfg), dtype=np.float64)
    P = net.unpack(cfg, theta)
    # spot-check that the oracle's unpacking lands on the layout's offsets
    for lname, shape, kind, off, n in param_layout(cfg):
        if lname == "pos_emb":
            assert P["pos"].ravel()[0] == off
        if lname == "l0.codebook":
            assert P["layers"][0]["codebook"].ravel()[0] == off
        if lname == "W_head":
            assert P["W_head"].ravel()[0] == off


def test_autoregressive_normalisation():
    cfg = CONFIGS["small"]
    P = net.unpack(cfg, make_params(cfg, std=0.5))
    lp = net.logpsi_fn(cfg, P, chunk=8192)(all_configs(cfg.N))
    total = np.exp(2.0 * lp).sum()
    assert abs(total - 1.0) < 1e-12


def test_conditionals_normalised_per_position():
    cfg = CONFIGS["small"]
    P = net.unpack(cfg, make_params(cfg))
    out = net.forward(cfg, P, make_spins(cfg, batch=32))
    assert np.allclose(np.exp(out["lp"]).sum(axis=-1), 1.0, atol=1e-14)


def test_causal_prefix_invariance():
    cfg = with_batch(CONFIGS["medium"], 4)
    P = net.unpack(cfg, make_params(cfg))
    s = make_spins(cfg)
    rng = np.random.default_rng(7)
    for b in range(4):
        j = int(rng.integers(1, cfg.N))
        s2 = s[b].copy()
        s2[j:] = -s2[j:]
        o1 = net.forward(cfg, P, s[b:b + 1])
        o2 = net.forward(cfg, P, s2[None])
        # positions < j see the same inputs and targets
        assert np.allclose(o1["ell"][0, :j], o2["ell"][0, :j], rtol=0,
                           atol=1e-13)
        assert (o1["codes"][:, 0, :j] == o2["codes"][:, 0, :j]).all()
        # and the target at j itself flips, with the same hidden state
        assert np.allclose(o1["lp"][0, j], o2["lp"][0, j], atol=1e-13)


def test_layer_norm_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 7, 32)) * 3 + 1
    g, b = rng.standard_normal(32), rng.standard_normal(32)
    ref = F.layer_norm(torch.tensor(x), (32,), torch.tensor(g),
                       torch.tensor(b), eps=1e-5).numpy()
    assert np.allclose(net.layer_norm(x, g, b), ref, rtol=1e-12, atol=1e-12)


def test_gelu_matches_torch_exact():
    x = np.linspace(-6, 6, 1001)
    ref = F.gelu(torch.tensor(x), approximate="none").numpy()
    assert np.allclose(net.gelu(x), ref, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("n_heads", [1, 2, 8])
def test_causal_attention_matches_torch_sdpa(n_heads):
    rng = np.random.default_rng(n_heads)
    S, N, d = 3, 20, 32
    q, k, v = (rng.standard_normal((S, N, d)) for _ in range(3))
    out = net.causal_attention(q, k, v, n_heads)

    def split(t):
        return torch.tensor(t).reshape(S, N, n_heads, d // n_heads).transpose(1, 2)

    ref = F.scaled_dot_product_attention(split(q), split(k), split(v),
                                         is_causal=True)
    ref = ref.transpose(1, 2).reshape(S, N, d).numpy()
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12)
    # subset of query rows gives the same rows
    rows = np.arange(7, N)
    sub = net.causal_attention(q[:, rows], k, v, n_heads, rows=rows)
    assert np.allclose(sub, out[:, rows], rtol=0, atol=1e-14)


def test_quantize_matches_bruteforce():
    rng = np.random.default_rng(3)
    H, Q, m = 4, 64, 8
    cb = rng.standard_normal((H, Q, m))
    a = rng.standard_normal((300, H * m))
    codes, z, d1, d2 = net.quantize(a, cb)
    for h in range(H):
        D = torch.cdist(torch.tensor(a[:, h * m:(h + 1) * m]),
                        torch.tensor(cb[h])).numpy()
        assert (codes[:, h] == D.argmin(axis=1)).all()
        Ds = np.sort(D, axis=1)
        assert np.allclose(d1[:, h], Ds[:, 0], rtol=1e-12)
        assert np.allclose(d2[:, h], Ds[:, 1], rtol=1e-12)
        assert np.array_equal(z[:, h * m:(h + 1) * m], cb[h][codes[:, h]])


def test_quantize_ties_and_exact_codewords():
    cb = np.array([[[1.0, 0.0], [0.0, 1.0], [1.0, 0.0], [-1.0, 0.0]]])
    a = np.array([[1.0, 0.0],      # exact codeword 0 (duplicated as 2)
                  [0.5, 0.5],      # equidistant to 0, 1, 2 -> lowest (0)
                  [-0.9, 0.1],     # nearest 3
                  [0.0, 0.9]])     # nearest 1
    codes, z, d1, d2 = net.quantize(a, cb)
    assert codes[:, 0].tolist() == [0, 0, 3, 1]
    assert d1[0, 0] == 0.0 and d2[0, 0] == 0.0
    # the paper's printed index formula is argmax over -distance, i.e. the
    # nearest code; the farthest code would have been 3, 3, 0, 3
    assert codes[2, 0] != 0


def test_head_permutation_invariance():
    cfg = with_batch(CONFIGS["medium"], 3)
    theta = make_params(cfg)
    s = make_spins(cfg)
    P = net.unpack(cfg, theta)
    lp1 = net.forward(cfg, P, s)["logpsi"]
    d, nh = cfg.d_model, cfg.n_heads
    dh = d // nh
    perm = np.array([2, 0, 3, 1])
    cols = np.concatenate([np.arange(p * dh, (p + 1) * dh) for p in perm])
    P2 = net.unpack(cfg, theta.copy())
    for lay in P2["layers"]:
        W, bq = lay["W_qkv"].copy(), lay["b_qkv"].copy()
        for part in range(3):
            lay["W_qkv"][:, part * d:(part + 1) * d] = W[:, part * d + cols]
            lay["b_qkv"][part * d:(part + 1) * d] = bq[part * d + cols]
        # attention output is permuted; VQ with one head sees a permuted
        # vector, so permute the codebook columns and W_o rows to match
        lay["codebook"][0] = lay["codebook"][0][:, cols].copy()
        lay["W_o"][:] = lay["W_o"][cols].copy()
    lp2 = net.forward(cfg, P2, s)["logpsi"]
    assert np.allclose(lp1, lp2, rtol=0, atol=1e-12)


def test_attention_tail_normalisation_and_causality():
    """A model ending with the attention-only half-block is still a
    normalised autoregressive distribution, and its conditionals at i do
    not depend on spins at or after i."""
    from dataclasses import replace
    cfg = replace(CONFIGS["small"], attn_tail=True)
    assert net.n_params(cfg) == param_count(cfg)
    P = net.unpack(cfg, make_params(cfg, std=0.5))
    assert "tail" in P
    lp = net.logpsi_fn(cfg, P, chunk=8192)(all_configs(cfg.N))
    assert abs(np.exp(2.0 * lp).sum() - 1.0) < 1e-12
    s = make_spins(cfg, batch=2)
    base = net.forward(cfg, P, s)["lp"]
    t = s.copy()
    t[:, 9:] = -t[:, 9:]
    assert np.array_equal(net.forward(cfg, P, t)["lp"][:, :10], base[:, :10])
