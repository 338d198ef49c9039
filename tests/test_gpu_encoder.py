"""The bidirectional encoder with mean pooling used as log psi (Sec. 3.1: the
encoder network pools its last layer's hidden states and maps them linearly
to a scalar) on the GPU against the FP64 oracle, through the C ABI.

* FP64 4x4, tokens of 1 and of 4 spins: log psi within 1e-12 of the
  oracle's forward pass; local energies of eq. (2) in the dedup form (every
  row attends again, the pooled mean is corrected over the changed rows)
  and in the plain form within 1e-10 of the oracle's plain re-evaluation,
  every ratio within 1e-10.
* FP64 4x4: the straight-through gradient of eqs. (7)-(8) within 1e-9 of the
  oracle's largest entry, per sample and weighted.
* FP64 chain of 10 sites: local energies of the transverse-field Ising
  chain within 1e-10.
* FP32 10x10, tokens of 4: every ratio within 1e-4 of the oracle or a proven
  near-tie; log psi within 1e-4 (or a proven near-tie) and the gradient of
  three samples per tensor within the FP32 bound.
* BF16 on the matrix core (6x6, d=128, tokens of 1 and of 4 spins): log
  psi within 1e-3 of the oracle on every sequence without a quantizer
  near-tie, the dedup form equal to the plain one, sampled ratios within
  1e-3 or proven near-ties, the gradient per tensor within the BF16 bound.
* BF16 on the matrix core, transverse-field Ising chains: 64 sites at head
  width 16 (open with tokens of 1, periodic with tokens of 4) and 32, and
  400 sites at head width 16 (two workgroups per CU): log psi within 1e-3
  or proven near-ties, dedup equal to plain, the local energy assembled as
  eq. (2) says, sampled flip ratios within 1e-3 or proven near-ties.
* Direct sampling and the VMC step need an autoregressive network: both
  report VQNQS_ERR_UNSUPPORTED for the encoder.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq
from oracle import eloc as oeloc
from oracle import grad as og
from oracle import lattice
from oracle import network as net
from oracle import tfim
from workloads import CONFIGS, make_params, make_spins, with_batch

from gpu_common import dev_params, dev_spins, host, needs_gpu, say
from gpu_parity import (BF16_BLOCK_TOL, FP32_BLOCK_TOL, check_blocks,
                        check_ratios, check_sequences)

pytestmark = [pytest.mark.gpu, needs_gpu]

ENC = replace(CONFIGS["small"], name="small_enc", encoder=True, batch=48,
              spin_seed=1012)
ENC4 = replace(ENC, name="small_enc_g4", group=4, spin_seed=1013)


@pytest.mark.parametrize("mc", [ENC, ENC4], ids=["K1", "K4"])
def test_encoder_fp64_forward_and_local_energy(mc):
    say(f"encoder fp64 {mc.name}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "f64"), dev_spins(s)
    lp = host(vq.forward_logpsi(cfg, p, sp))
    ref = net.forward(mc, net.unpack(mc, theta), s)["logpsi"]
    assert np.allclose(lp, ref, rtol=0, atol=1e-12)
    E_ref, r_ref = oeloc.eloc_network_naive(mc, theta, s, return_ratios=True)
    for mode in (vq.DEDUP, vq.PLAIN):
        out = vq.local_energy(cfg, p, sp, mode, ratios=True)
        E, R = host(out["eloc"]), host(out["ratios"])
        assert np.allclose(E, E_ref, rtol=1e-10, atol=0), mode
        for b in range(mc.batch):
            k = len(r_ref[b])
            assert np.allclose(R[b, :k], r_ref[b], rtol=1e-10, atol=0)
            assert (R[b, k:] == 0).all()


def test_encoder_fp64_gradient():
    mc = with_batch(ENC, 3)
    say("encoder fp64 gradient")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "f64"), dev_spins(s)
    g = host(vq.grad_logpsi(cfg, p, sp))
    ref = og.grad_logpsi(mc, theta, s)
    assert np.abs(g - ref).max() <= 1e-9 * np.abs(ref).max()
    w = np.array([0.25, -1.5, 1.0])
    gw = host(vq.grad_logpsi(cfg, p, sp, weights=torch.tensor(w, device="cuda")))
    assert np.abs(gw - w @ ref).max() <= 1e-9 * np.abs(w @ ref).max()


def test_encoder_tfim_fp64():
    mc = replace(CONFIGS["tfim_small"], name="tfim_enc", encoder=True,
                 batch=32)
    say("encoder tfim fp64")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "f64"), dev_spins(s)
    E_ref = tfim.eloc_network_naive(mc, theta, s)
    for mode in (vq.DEDUP, vq.PLAIN):
        E = host(vq.local_energy(cfg, p, sp, mode)["eloc"])
        assert np.allclose(E, E_ref, rtol=1e-10, atol=0), mode


def test_encoder_fp32_medium():
    mc = with_batch(replace(CONFIGS["medium"], name="medium_enc_g4",
                            encoder=True, group=4, precision="f32"), 8)
    say("encoder fp32 10x10 K=4")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p = dev_params(theta, "f32")
    R = host(vq.local_energy(cfg, p, dev_spins(s), vq.DEDUP, ratios=True)["ratios"])
    bl = lattice.bonds(mc.L, mc.periodic)
    picks = [(b, range(len(lattice.neighbours(s[b], bl)))) for b in range(mc.batch)]
    rel, explained = check_ratios(mc, net.unpack(mc, theta), cfg, p, s, R,
                                  picks, 1e-4)
    say(f"encoder fp32 ratios: median {np.median(rel):.2e} max {rel.max():.2e}, "
        f"{len(explained)} explained")
    g = host(vq.grad_logpsi(cfg, p, dev_spins(s))).astype(np.float64)
    flips, _ = check_sequences(mc, net.unpack(mc, theta), cfg, p, s, 1e-4)
    idx = [b for b in range(mc.batch) if b not in flips][:3]
    assert idx
    ref = og.grad_logpsi(mc, theta, s[idx])
    for j, b in enumerate(idx):
        check_blocks(mc, g[b], ref[j], FP32_BLOCK_TOL, f"encoder fp32 sample {b}")


def test_encoder_sampling_and_vmc_rejected():
    mc = with_batch(ENC, 4)
    cfg = vq.make_config(mc)
    p = dev_params(make_params(mc), "f64")
    u = torch.rand((mc.batch, mc.N), dtype=torch.float64, device="cuda")
    with pytest.raises(vq.VQNQSError) as e:
        vq.sample(cfg, p, u)
    assert e.value.status == 5
    with pytest.raises(vq.VQNQSError) as e:
        vq.vmc_step(cfg, p, u, 1e-3)
    assert e.value.status == 5


@pytest.mark.parametrize("group", [1, 4], ids=["K1", "K4"])
def test_encoder_bf16_matrix_core(group):
    mc = replace(CONFIGS["small"], name=f"enc_bf16_g{group}", L=6, d_model=128,
                 n_layers=2, n_heads=8, d_ff=512, codebook_size=64,
                 precision="bf16", encoder=True, group=group, batch=12,
                 spin_seed=1801 + group)
    say(f"encoder bf16 6x6 K={group}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    P = net.unpack(mc, theta)
    flips, _ = check_sequences(mc, P, cfg, p, s, 1e-3)
    a = vq.local_energy(cfg, p, sp, vq.PLAIN, ratios=True)
    b = vq.local_energy(cfg, p, sp, vq.DEDUP, ratios=True)
    assert np.allclose(host(b["ratios"]), host(a["ratios"]), rtol=1e-12, atol=0)
    R = host(b["ratios"])
    bl = lattice.bonds(mc.L, mc.periodic)
    picks = [(k, range(len(lattice.neighbours(s[k], bl)))) for k in range(4)]
    rel, explained = check_ratios(mc, P, cfg, p, s, R, picks, 1e-3)
    say(f"encoder bf16 ratios: median {np.median(rel):.2e} max {rel.max():.2e}, "
        f"{len(explained)} explained")
    g = host(vq.grad_logpsi(cfg, p, sp)).astype(np.float64)
    idx = [k for k in range(mc.batch) if k not in flips][:3]
    assert idx
    ref = og.grad_logpsi(mc, theta, s[idx])
    for j, k in enumerate(idx):
        check_blocks(mc, g[k], ref[j], BF16_BLOCK_TOL, f"encoder bf16 sample {k}")


# (sites, width, tokens of K, periodic): head width 16 with three
# workgroups per CU, head width 32, and head width 16 at 400 tokens, whose
# LDS tiles leave room for two workgroups per CU (the uncapped kernel)
CHAINS = [(64, 128, 1, False), (64, 128, 4, True), (64, 256, 1, True),
          (400, 128, 1, False)]


@pytest.mark.parametrize("L,d,group,periodic", CHAINS,
                         ids=["64-dh16-K1-open", "64-dh16-K4-periodic",
                              "64-dh32-K1-periodic", "400-dh16-K1-open"])
def test_encoder_bf16_tfim_chain(L, d, group, periodic):
    mc = replace(CONFIGS["tfim"], name=f"enc_tfim_bf16_{L}_{d}_g{group}", L=L,
                 d_model=d, n_layers=2, d_ff=4 * d, encoder=True, group=group,
                 periodic=periodic, batch=16 if L <= 64 else 6,
                 spin_seed=1811 + group + L + d)
    say(f"encoder bf16 chain of {L} d={d} K={group} periodic={periodic}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    P = net.unpack(mc, theta)
    check_sequences(mc, P, cfg, p, s, 1e-3)
    a = vq.local_energy(cfg, p, sp, vq.PLAIN, ratios=True)
    b = vq.local_energy(cfg, p, sp, vq.DEDUP, ratios=True)
    assert np.allclose(host(b["ratios"]), host(a["ratios"]), rtol=1e-12, atol=0)
    E, R = host(b["eloc"]), host(b["ratios"])
    diag = tfim.diagonal(s, mc.N, periodic, mc.J)
    assert np.allclose(E, diag - mc.gamma * R[:, :mc.N].sum(1), rtol=1e-12,
                       atol=1e-12)
    rng = np.random.default_rng(group)
    picks = [(k, sorted(rng.choice(mc.N, 12, replace=False))) for k in range(3)]
    rel, explained = check_ratios(mc, P, cfg, p, s, R, picks, 1e-3)
    say(f"encoder bf16 chain ratios: median {np.median(rel):.2e} "
        f"max {rel.max():.2e}, {len(explained)} explained")
