"""GPU parity of the straight-through gradient of log psi (eqs. 7-8)
against the FP64 oracle, through the C ABI.

FP64: per-sample and weighted gradients within 1e-9 of the largest entry
(the two sides add in different orders; distances are expanded on the GPU
and taken directly in the oracle).  FP32 and BF16: every parameter tensor
(each embedding, LayerNorm gain and bias, weight matrix, bias and codebook
of every layer, and the head) separately, its largest entry error within
FP32_BLOCK_TOL = 1e-4 (FP32) or BF16_BLOCK_TOL = 1e-2 (BF16; the forward
and its recompute run on the matrix core at the hi/lo split's 2^-17) of
that tensor's largest entry, so an error in a small tensor cannot hide in
the norm of the whole vector.  In BF16 the forward decides codes in its own
precision: samples whose codes all equal the oracle's are compared, and a
sample with a differing code must be a proven near-tie
(tests/near_tie.py)."""
from dataclasses import replace

import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq
from oracle import grad as og
from oracle import network as net
from workloads import CONFIGS, make_params, make_spins, with_batch

from gpu_common import dev_params, dev_spins, host, needs_gpu, say
from gpu_parity import (BF16_BLOCK_TOL, FP32_BLOCK_TOL, check_blocks,
                         check_sequences)

pytestmark = [pytest.mark.gpu, needs_gpu]

TWO_VQ = replace(CONFIGS["small"], name="two_vq", L=4, d_model=8,
                 n_layers=2, n_heads=2, d_ff=16, codebook_size=6, vq_heads=2,
                 batch=3, spin_seed=1701)


def rel_max(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def rel_norm(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)



@pytest.mark.parametrize("mc", [with_batch(CONFIGS["small"], 4), TWO_VQ,
                                with_batch(CONFIGS["medium"], 2,
                                           precision="f64")],
                         ids=["small", "two_vq", "medium"])
def test_grad_f64_per_sample_and_weighted(mc):
    say(f"grad f64 {mc.name} B={mc.batch}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "f64"), dev_spins(s)
    g, lp = vq.grad_logpsi(cfg, p, sp, logpsi=True)
    ref = og.grad_logpsi(mc, theta, s)
    assert rel_max(host(g), ref) < 1e-9
    ref_lp = net.forward(mc, net.unpack(mc, theta), s)["logpsi"]
    assert np.allclose(host(lp), ref_lp, rtol=1e-12, atol=1e-12)
    w = np.linspace(-1.0, 2.0, mc.batch)
    gw = vq.grad_logpsi(cfg, p, sp, weights=torch.tensor(w, device="cuda"))
    assert rel_max(host(gw), w @ ref) < 1e-9


Q2_W1 = replace(CONFIGS["small"], name="q2_w1", L=4, d_model=4, n_layers=2,
                n_heads=1, d_ff=8, codebook_size=2, vq_heads=4, batch=3,
                spin_seed=1703)
Q3_W2 = replace(CONFIGS["small"], name="q3_w2", L=4, d_model=4, n_layers=2,
                n_heads=1, d_ff=8, codebook_size=3, vq_heads=2, batch=3,
                spin_seed=1707)


@pytest.mark.parametrize("mc", [Q2_W1, Q3_W2], ids=["q2_w1", "q3_w2"])
def test_grad_f64_small_quantizers(mc):
    """The quantizers of the oracle's closed-form pins of eq. (8) (two
    codewords of width 1; three codewords of width 2, two heads) inside a
    whole network, FP64 through the C ABI, per sample and weighted."""
    say(f"grad f64 {mc.name}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "f64"), dev_spins(s)
    g = host(vq.grad_logpsi(cfg, p, sp))
    ref = og.grad_logpsi(mc, theta, s)
    assert rel_max(g, ref) < 1e-9
    w = np.array([0.25, -1.5, 1.0])
    gw = host(vq.grad_logpsi(cfg, p, sp, weights=torch.tensor(w, device="cuda")))
    assert rel_max(gw, w @ ref) < 1e-9


def test_grad_f32_medium():
    mc = with_batch(CONFIGS["medium"], 2)
    say("grad f32 medium")
    theta = make_params(mc)
    s = make_spins(mc)
    g = vq.grad_logpsi(vq.make_config(mc), dev_params(theta, "f32"),
                       dev_spins(s))
    ref = og.grad_logpsi(mc, theta, s)
    G = host(g).astype(np.float64)
    for b in range(mc.batch):
        check_blocks(mc, G[b], ref[b], FP32_BLOCK_TOL, f"fp32 sample {b}")


def test_grad_bf16_grad_shapes_sampled():
    """The 20x20 gradient workload's model (d=256, 12 layers, 8 heads, MLP
    1024, Q=1024) on a few seeded samples, recomputed one by one by the
    oracle."""
    mc = with_batch(CONFIGS["grad"], 6)
    say("grad bf16 20x20 sampled")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    g = host(vq.grad_logpsi(cfg, p, sp)).astype(np.float64)
    flips, _ = check_sequences(mc, net.unpack(mc, theta), cfg, p, s, 1e-3)
    idx = [b for b in range(mc.batch) if b not in flips][:2]
    assert len(idx) >= 1
    ref = og.grad_logpsi(mc, theta, s[idx])
    for j, b in enumerate(idx):
        check_blocks(mc, g[b], ref[j], BF16_BLOCK_TOL, f"bf16 sample {b}")


def test_grad_bf16_chain_four_quantizer_heads():
    """The paper's chain network (384 sites, d=256, one layer, 8 heads, a
    quantizer of 4 heads x 64 codes): the straight-through gradient with
    several quantizer heads, per tensor against the oracle."""
    mc = with_batch(CONFIGS["tfim"], 4)
    assert mc.vq_heads == 4 and mc.precision == "bf16"
    say("grad bf16 chain of 384, 4 quantizer heads")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    g = host(vq.grad_logpsi(cfg, p, sp)).astype(np.float64)
    flips, _ = check_sequences(mc, net.unpack(mc, theta), cfg, p, s, 1e-3)
    idx = [b for b in range(mc.batch) if b not in flips][:2]
    assert len(idx) >= 1
    ref = og.grad_logpsi(mc, theta, s[idx])
    for j, b in enumerate(idx):
        check_blocks(mc, g[b], ref[j], BF16_BLOCK_TOL, f"bf16 chain sample {b}")


ODD_BF16 = replace(CONFIGS["medium"], name="odd_bf16", L=5, periodic=False,
                   d_model=64, n_layers=2, n_heads=4, d_ff=256,
                   codebook_size=64, precision="bf16", batch=3, spin_seed=2024)


def test_grad_bf16_row_count_not_multiple_of_four():
    """Open 5x5 lattice, 3 samples: 75 rows, so the matrix-core products see
    row ranges that end inside a 4-row block (the guarded element loads)
    besides the 16-byte ones; checked against the oracle like the 20x20
    case."""
    mc = ODD_BF16
    say("grad bf16 odd rows")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    g = host(vq.grad_logpsi(cfg, p, sp)).astype(np.float64)
    flips, _ = check_sequences(mc, net.unpack(mc, theta), cfg, p, s, 1e-3)
    idx = [b for b in range(mc.batch) if b not in flips]
    assert len(idx) >= 1
    ref = og.grad_logpsi(mc, theta, s[idx])
    for j, b in enumerate(idx):
        check_blocks(mc, g[b], ref[j], BF16_BLOCK_TOL, f"bf16 odd sample {b}")
    w = torch.linspace(-1.0, 1.0, mc.batch, dtype=torch.float64, device="cuda")
    gw = host(vq.grad_logpsi(cfg, p, sp, weights=w)).astype(np.float64)
    assert rel_norm(gw, host(w) @ g) < 1e-5


def test_grad_autograd_function_matches_weighted():
    mc = with_batch(CONFIGS["small"], 5)
    say("grad autograd function")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p = dev_params(theta, "f64").requires_grad_(True)
    w = torch.linspace(0.5, -1.5, mc.batch, dtype=torch.float64, device="cuda")
    (w * vq.logpsi(cfg, p, dev_spins(s))).sum().backward()
    gw = vq.grad_logpsi(cfg, p.detach(), dev_spins(s), weights=w)
    assert np.array_equal(host(p.grad), host(gw))


def test_grad_chunking_and_repeat_bitwise():
    mc = with_batch(CONFIGS["small"], 7)
    say("grad chunking")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "f64"), dev_spins(s)
    w = torch.linspace(-1.0, 1.0, mc.batch, dtype=torch.float64, device="cuda")
    full = host(vq.grad_logpsi(cfg, p, sp, weights=w))
    again = host(vq.grad_logpsi(cfg, p, sp, weights=w))
    small = torch.empty(vq.workspace_size(cfg, mc.batch, vq.WS_GRAD, 3),
                        dtype=torch.uint8, device="cuda")
    chunked = host(vq.grad_logpsi(cfg, p, sp, weights=w, ws=small))
    assert np.array_equal(full, again)
    assert np.array_equal(full, chunked)
    per = host(vq.grad_logpsi(cfg, p, sp))
    per_c = host(vq.grad_logpsi(cfg, p, sp, ws=small))
    assert np.array_equal(per, per_c)


def test_grad_empty_batch_weighted_is_zero():
    mc = CONFIGS["small"]
    cfg = vq.make_config(mc)
    theta = make_params(mc)
    p = dev_params(theta, "f64")
    sp = torch.empty((0, mc.N), dtype=torch.int8, device="cuda")
    g = vq.grad_logpsi(cfg, p, sp, weights=torch.empty(0, dtype=torch.float64,
                                                       device="cuda"))
    assert g.shape == (p.numel(),)
    assert not host(g).any()
