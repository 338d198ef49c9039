"""Whole-network pins of the oracle's forward pass (CPU only): parameter
choices under which the VQ transformer of Sec. 3.1 reduces to a closed form
built from library routines (torch LayerNorm, exact GELU, log-softmax,
cumulative sums, torch.cdist), so that the composition of the blocks is
checked, not only each operation on its own.

* Pass-through blocks: with the output projection and the second MLP
  matrix and their biases at zero, every block (and the attention-only
  half-block) is the identity, and log psi is the head alone on the
  embedded shifted tokens: 1/2 sum_i log softmax(LN(tok[u_i] + pos_i) W + b)
  at the target token.  Pins the residual form, the input shift with the
  beginning-of-sequence token 2^K, tokens of K spins, the position
  embedding, the final LN, the head and the factor 1/2 of the polar form
  (Sec. 2).
* Uniform attention: with the query and key projections at zero every
  score is zero, so causal attention is the running mean of the values
  over keys j <= i (every key in the encoder).  The rest of each block is
  then evaluated from its description in Sec. 3.1 with library routines:
  pre-LN, quantizer on the attention output before W_o (nearest codeword
  per segment by torch.cdist), residual, MLP on LN2 of the updated stream,
  residual.  Pins the causal direction of the mask (the diagonal
  included), the value path, the quantizer's place in the block and the
  order of the two sub-blocks; for the encoder also attention over every
  key and mean pooling after the final LN (Sec. 3.1).

A dropped residual, a mask that excludes the diagonal or looks ahead, LN2
applied to the block input instead of the updated stream, the quantizer
after W_o, or a missing shift each change log psi by far more than the
1e-12 these tests allow.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import network as net
from workloads import CONFIGS, make_params, make_spins

EPS = 1e-5


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


def _ln(x, g, b):
    return F.layer_norm(_t(x), (x.shape[-1],), _t(g), _t(b), eps=EPS).numpy()


def _gelu(x):
    return F.gelu(_t(x), approximate="none").numpy()


def _log_softmax(x):
    return torch.log_softmax(_t(x), dim=-1).numpy()


def _token_ids(spins, K):
    """Target tokens and shifted inputs, built bit by bit from the spins:
    the k-th site of a token contributes 2^k when it holds spin -1."""
    S, N = spins.shape
    T = N // K
    t = np.zeros((S, T), dtype=np.int64)
    for i in range(T):
        for k in range(K):
            t[:, i] += np.where(spins[:, i * K + k] < 0, 1 << k, 0)
    u = np.empty_like(t)
    u[:, 0] = 1 << K
    u[:, 1:] = t[:, :-1]
    return t, u


def _nearest_vq(a, codebook):
    """Nearest codeword per segment by brute force (torch.cdist)."""
    H, Q, m = codebook.shape
    z = np.empty_like(a)
    codes = np.empty(a.shape[:-1] + (H,), dtype=np.int64)
    flat = a.reshape(-1, a.shape[-1])
    zf = z.reshape(-1, a.shape[-1])
    cf = codes.reshape(-1, H)
    for h in range(H):
        seg = _t(flat[:, h * m:(h + 1) * m])
        dist = torch.cdist(seg, _t(codebook[h]))
        c = torch.argmin(dist, dim=1).numpy()
        cf[:, h] = c
        zf[:, h * m:(h + 1) * m] = codebook[h][c]
    return codes, z


def _running_mean(v, causal):
    """Attention with all scores equal: the mean of the values over the
    keys each query sees."""
    if not causal:
        return np.broadcast_to(v.mean(axis=-2, keepdims=True), v.shape).copy()
    n = np.arange(1, v.shape[-2] + 1, dtype=np.float64)[:, None]
    return torch.cumsum(_t(v), dim=-2).numpy() / n


def _config(K, tail=False, encoder=False):
    return replace(CONFIGS["small"], name=f"cf_K{K}", group=K,
                   attn_tail=tail, encoder=encoder, batch=24,
                   spin_seed=4100 + K)


@pytest.mark.parametrize("K,tail", [(1, False), (2, False), (1, True),
                                    (4, True)])
def test_pass_through_blocks_reduce_to_the_head(K, tail):
    cfg = _config(K, tail)
    theta = make_params(cfg, std=0.4)
    P = net.unpack(cfg, theta)
    for lay in P["layers"]:
        for key in ("W_o", "b_o", "W2", "b2"):
            lay[key][...] = 0.0
    if tail:
        P["tail"]["W_o"][...] = 0.0
        P["tail"]["b_o"][...] = 0.0
    spins = make_spins(cfg)
    t, u = _token_ids(spins, K)
    x = P["tok"][u] + P["pos"][None]
    lp = _log_softmax(_ln(x, P["lnf_g"], P["lnf_b"]) @ P["W_head"]
                      + P["b_head"])
    ref = 0.5 * np.take_along_axis(lp, t[..., None], axis=-1)[..., 0].sum(-1)
    got = net.forward(cfg, P, spins)["logpsi"]
    assert np.allclose(got, ref, rtol=0, atol=1e-12)
    # the same parameters with the output projection restored differ: the
    # blocks are not trivially skipped
    P2 = net.unpack(cfg, make_params(cfg, std=0.4))
    assert np.abs(net.forward(cfg, P2, spins)["logpsi"] - ref).max() > 1e-3


def _uniform_attention_params(cfg, std=0.4):
    P = net.unpack(cfg, make_params(cfg, std=std))
    d = cfg.d_model
    blocks = list(P["layers"]) + ([P["tail"]] if "tail" in P else [])
    for lay in blocks:
        lay["W_qkv"][:, :2 * d] = 0.0
        lay["b_qkv"][:2 * d] = 0.0
    return P


def _blocks_closed_form(cfg, P, x, causal):
    d = cfg.d_model
    codes = []
    for lay in P["layers"]:
        h = _ln(x, lay["ln1_g"], lay["ln1_b"])
        v = h @ lay["W_qkv"][:, 2 * d:] + lay["b_qkv"][2 * d:]
        a = _running_mean(v, causal)
        c, z = _nearest_vq(a, lay["codebook"])
        codes.append(c)
        xp = x + z @ lay["W_o"] + lay["b_o"]
        x = xp + _gelu(_ln(xp, lay["ln2_g"], lay["ln2_b"]) @ lay["W1"]
                       + lay["b1"]) @ lay["W2"] + lay["b2"]
    if "tail" in P:
        T = P["tail"]
        v = _ln(x, T["ln_g"], T["ln_b"]) @ T["W_qkv"][:, 2 * d:] + T["b_qkv"][2 * d:]
        x = x + _running_mean(v, causal) @ T["W_o"] + T["b_o"]
    return x, np.stack(codes)


@pytest.mark.parametrize("K,tail", [(1, False), (2, True), (4, False)])
def test_uniform_attention_decoder(K, tail):
    cfg = _config(K, tail)
    P = _uniform_attention_params(cfg)
    spins = make_spins(cfg)
    t, u = _token_ids(spins, K)
    x, codes = _blocks_closed_form(cfg, P, P["tok"][u] + P["pos"][None],
                                   causal=True)
    lp = _log_softmax(_ln(x, P["lnf_g"], P["lnf_b"]) @ P["W_head"]
                      + P["b_head"])
    ref = 0.5 * np.take_along_axis(lp, t[..., None], axis=-1)[..., 0].sum(-1)
    out = net.forward(cfg, P, spins)
    assert np.array_equal(out["codes"], codes)
    assert np.allclose(out["logpsi"], ref, rtol=0, atol=1e-12)
    # more than one code per layer is in use, so the quantizer decides
    assert all(len(np.unique(c)) > 1 for c in codes)


@pytest.mark.parametrize("K", [1, 2, 4])
def test_uniform_attention_encoder(K):
    cfg = _config(K, encoder=True)
    P = _uniform_attention_params(cfg)
    spins = make_spins(cfg)
    t, _ = _token_ids(spins, K)
    x, codes = _blocks_closed_form(cfg, P, P["tok"][t] + P["pos"][None],
                                   causal=False)
    f = _ln(x, P["lnf_g"], P["lnf_b"])
    ref = (f @ P["W_head"])[..., 0].mean(-1) + P["b_head"][0]
    out = net.forward(cfg, P, spins)
    assert np.array_equal(out["codes"], codes)
    assert np.allclose(out["logpsi"], ref, rtol=0, atol=1e-12)
