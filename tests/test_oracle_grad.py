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
  and the codebook receives twice the true derivative (one-hot path plus
  softmax path, both kept by the literal eq. 8).
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
        assert abs(2 * fd - g[i]) <= 1e-7 * (1 + abs(fd)), (i, fd, g[i])


def test_weighted_equals_sum_of_per_sample():
    cfg = SMALL
    th = make_params(cfg)
    s = make_spins(cfg)
    w = np.array([0.5, -1.25, 2.0])
    G = og.grad_logpsi(cfg, th, s)
    gw = og.grad_logpsi(cfg, th, s, weights=w)
    assert np.allclose(gw, w @ G, rtol=1e-12, atol=1e-12)
