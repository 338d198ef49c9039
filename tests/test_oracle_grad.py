"""Pins of the straight-through gradient oracle (eqs. 7-8).

* The surrogate's value is the forward pass of the network oracle.
* Central finite differences of the surrogate (codes and subtracted soft
  values frozen at theta0) equal its autograd gradient along random
  directions.
* Parameters after the last quantizer see a smooth network: there the
  straight-through gradient is the true derivative, checked by central
  differences of the NumPy forward pass (independent code).
* One codeword per head (Q = 1): the softmax is constant, so no gradient
  reaches anything that only feeds the quantizer (LN1, QKV of every layer),
  and the codebook receives exactly the true derivative: in eq. (8) the
  codebook factor of g(D)^T W is multiplied by the value of g, the one-hot
  vector, and the softmax term contributes nothing when p is constant.
* Closed forms of eq. (8) on a single quantizer, derived by hand (not by
  autograd): two codewords on a line, W1 < u < W2, where
  p = softmax(-(u - W1), -(W2 - u)) gives dV/du = 2 p1 p2 (W2 - W1) and
  dV/dW_j = [j = c] - p1 p2 (W2 - W1); and three codewords in the plane
  with two quantizer heads at a generic point, against the chain rule
  through the unsquared distances written out in NumPy.  A softmax of +D,
  a squared distance, a dropped softmax path or a softmax term on the
  codebook factor each fail one of these.
* Weighted and per-sample forms agree.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import grad as og
from oracle import network as onet
from workloads import CONFIGS, make_params, make_spins, with_batch
from workloads.layout import param_layout

SMALL = with_batch(CONFIGS["small"], 3)
TINY2 = replace(CONFIGS["small"], name="tiny2", L=4, d_model=8, n_layers=2,
                n_heads=2, d_ff=16, codebook_size=6, vq_heads=2, batch=2)


def _slices(cfg, pred):
    idx = []
    for name, shape, kind, off, n in param_layout(cfg):
        if pred(name):
            idx.append(np.arange(off, off + n))
    return np.concatenate(idx)


@pytest.mark.parametrize("cfg", [SMALL, TINY2])
def test_surrogate_value_equals_forward(cfg):
    th = make_params(cfg)
    s = make_spins(cfg)
    ref = onet.forward(cfg, onet.unpack(cfg, th), s)["logpsi"]
    assert np.allclose(og.logpsi(cfg, th, s), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("cfg", [SMALL, TINY2])
def test_central_differences_of_surrogate(cfg):
    th = make_params(cfg)
    s = make_spins(cfg)[:1]
    g = og.grad_logpsi(cfg, th, s)[0]
    fr = og.frozen_state(cfg, th, s)
    rng = np.random.default_rng(5)
    eps = 1e-6
    for _ in range(4):
        v = rng.standard_normal(th.size)
        v /= np.linalg.norm(v)
        fp = og.surrogate_logpsi(cfg, th + eps * v, s, fr)[0]
        fm = og.surrogate_logpsi(cfg, th - eps * v, s, fr)[0]
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g @ v) <= 1e-7 * (1 + abs(fd)), (fd, g @ v)


def test_post_quantizer_gradient_is_true_derivative():
    cfg = TINY2
    th = make_params(cfg)
    s = make_spins(cfg)[:1]
    g = og.grad_logpsi(cfg, th, s)[0]
    last = cfg.n_layers - 1
    idx = _slices(cfg, lambda n: n.startswith(f"l{last}.") and
                  n.split(".")[-1] not in ("ln1_g", "ln1_b", "W_qkv", "b_qkv",
                                           "codebook")
                  or n in ("lnf_g", "lnf_b", "W_head", "b_head"))
    rng = np.random.default_rng(7)
    pick = rng.choice(idx, 40, replace=False)
    f = lambda t: onet.forward(cfg, onet.unpack(cfg, t), s)["logpsi"][0]
    eps = 1e-6
    for i in pick:
        e = np.zeros_like(th)
        e[i] = eps
        fd = (f(th + e) - f(th - e)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * (1 + abs(fd)), (i, fd, g[i])


def test_attention_tail_gradient_is_true_derivative():
    """The attention-only half-block has no quantizer: its parameters (and
    the final LayerNorm and head) get the true derivative, checked by
    central differences of the NumPy forward."""
    cfg = replace(TINY2, attn_tail=True)
    th = make_params(cfg)
    s = make_spins(cfg)[:1]
    g = og.grad_logpsi(cfg, th, s)[0]
    idx = _slices(cfg, lambda n: n.startswith("tail.")
                  or n in ("lnf_g", "lnf_b", "W_head", "b_head"))
    rng = np.random.default_rng(8)
    pick = rng.choice(idx, 40, replace=False)
    f = lambda t: onet.forward(cfg, onet.unpack(cfg, t), s)["logpsi"][0]
    eps = 1e-6
    for i in pick:
        e = np.zeros_like(th)
        e[i] = eps
        fd = (f(th + e) - f(th - e)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * (1 + abs(fd)), (i, fd, g[i])


def test_single_codeword_closed_forms():
    cfg = replace(TINY2, codebook_size=1)
    th = make_params(cfg)
    s = make_spins(cfg)[:1]
    g = og.grad_logpsi(cfg, th, s)[0]
    feeds_vq_only = _slices(cfg, lambda n: n.split(".")[-1] in
                            ("ln1_g", "ln1_b", "W_qkv", "b_qkv"))
    assert np.all(g[feeds_vq_only] == 0.0)
    cb = _slices(cfg, lambda n: n.endswith("codebook"))
    f = lambda t: onet.forward(cfg, onet.unpack(cfg, t), s)["logpsi"][0]
    eps = 1e-6
    for i in cb[::3]:
        e = np.zeros_like(th)
        e[i] = eps
        fd = (f(th + e) - f(th - e)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * (1 + abs(fd)), (i, fd, g[i])


def _st_grads(a, codebook, up):
    """Gradients of sum(up * z) for the oracle's quantizer z(a, W)."""
    import torch
    at = torch.tensor(a, dtype=torch.float64, requires_grad=True)
    wt = torch.tensor(codebook, dtype=torch.float64, requires_grad=True)
    z, codes, _ = og.vq_surrogate(at, wt)
    (z * torch.tensor(up, dtype=torch.float64)).sum().backward()
    grad = lambda t: (np.zeros(t.shape) if t.grad is None
                      else t.grad.numpy())
    return z.detach().numpy(), codes, grad(at), grad(wt)


@pytest.mark.parametrize("u", [-0.7, -0.1, 0.05, 0.3, 1.1])
def test_two_codewords_on_a_line_closed_form(u):
    """Eq. (8) with Q = 2, segment width 1, W1 = -0.8 < u < W2 = 1.3."""
    W1, W2, g = -0.8, 1.3, 0.6
    p1 = np.exp(-(u - W1)) / (np.exp(-(u - W1)) + np.exp(-(W2 - u)))
    p2 = 1.0 - p1
    c = 0 if (u - W1) <= (W2 - u) else 1
    z, codes, da, dW = _st_grads(np.array([[[u]]]),
                                 np.array([[[W1], [W2]]]), np.array([[[g]]]))
    assert codes[0, 0] == c
    assert z[0, 0, 0] == (W1, W2)[c]
    k = p1 * p2 * (W2 - W1)
    assert abs(da[0, 0, 0] - g * 2 * k) <= 1e-14
    assert abs(dW[0, 0, 0] - g * ((c == 0) - k)) <= 1e-14
    assert abs(dW[0, 1, 0] - g * ((c == 1) - k)) <= 1e-14


def test_three_codewords_two_heads_closed_form():
    """Eq. (8) with Q = 3, segment width 2, two quantizer heads, at a
    generic point; expected values from the chain rule through
    D_j = -||u - W_j||: with t_j = p_j (e_j - p.e), e_j = g . W_j,
        dL/du   = -sum_j t_j (u - W_j) / ||u - W_j||,
        dL/dW_j = [j = c] g + t_j (u - W_j) / ||u - W_j||."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal((2, 3, 4))           # S=2, N=3, d=4, H=2
    W = rng.standard_normal((2, 3, 2))
    up = rng.standard_normal((2, 3, 4))
    z, codes, da, dW = _st_grads(a, W, up)
    exp_da = np.zeros_like(a)
    exp_dW = np.zeros_like(W)
    for s in range(2):
        for i in range(3):
            for h in range(2):
                u = a[s, i, 2 * h:2 * h + 2]
                g = up[s, i, 2 * h:2 * h + 2]
                dist = np.array([np.sqrt(((u - W[h, j]) ** 2).sum())
                                 for j in range(3)])
                c = int(np.argmin(dist))
                assert codes[s * 3 + i, h] == c
                assert np.array_equal(z[s, i, 2 * h:2 * h + 2], W[h, c])
                p = np.exp(-dist) / np.exp(-dist).sum()
                e = np.array([g @ W[h, j] for j in range(3)])
                t = p * (e - p @ e)
                for j in range(3):
                    unit = (u - W[h, j]) / dist[j]
                    exp_da[s, i, 2 * h:2 * h + 2] -= t[j] * unit
                    exp_dW[h, j] += t[j] * unit + (j == c) * g
    assert np.allclose(da, exp_da, rtol=0, atol=1e-13)
    assert np.allclose(dW, exp_dW, rtol=0, atol=1e-13)


def test_weighted_equals_sum_of_per_sample():
    cfg = SMALL
    th = make_params(cfg)
    s = make_spins(cfg)
    w = np.array([0.5, -1.25, 2.0])
    G = og.grad_logpsi(cfg, th, s)
    gw = og.grad_logpsi(cfg, th, s, weights=w)
    assert np.allclose(gw, w @ G, rtol=1e-12, atol=1e-12)
