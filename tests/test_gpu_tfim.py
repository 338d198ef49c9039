"""The transverse-field Ising chain (Sec. 4) on the GPU against the FP64
oracle (oracle/tfim.py), through the C ABI.

* Neighbours: every site's flip, listed by site, and the exact diagonal
  -J sum s_i s_{i+1} (open and periodic chains).
* FP64 10-site chain: local energies of eq. (2) in the deduplicated and the
  plain form within 1e-10 of the oracle's plain re-evaluation, every ratio
  within 1e-10 (open and periodic).
* BF16, the paper's 384-site open chain (d=256, 1 layer, 8 heads, 4 x 64
  codes) at the full batch of 2048 in one call: seeded samples' ratios
  within 1e-3 of the oracle or proven near-ties, the local energy assembled
  as eq. (2) says; dedup equal to plain on a small batch.
* FP64 VMC step on the chain equal to the oracle's step (gradient descent).
"""
import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq
from oracle import tfim
from oracle import network as net
from oracle import sampling
from oracle import grad as ograd
from workloads import CONFIGS, make_params, make_spins, with_batch

from gpu_common import dev_params, dev_spins, host, needs_gpu, say
from gpu_parity import check_ratios

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.mark.parametrize("periodic", [False, True])
def test_tfim_neighbours_and_diagonal(periodic):
    mc = with_batch(CONFIGS["tfim_small"], 32, periodic=periodic, J=0.8)
    s = make_spins(mc)
    bonds, count, diag = vq.neighbours(vq.make_config(mc), dev_spins(s))
    bonds, count, diag = host(bonds), host(count), host(diag)
    assert (count == mc.N).all()
    assert (bonds[:, :mc.N] == np.arange(mc.N)).all()
    assert (bonds[:, mc.N:] == -1).all()
    assert np.array_equal(diag, tfim.diagonal(s, mc.N, periodic, mc.J))


@pytest.mark.parametrize("periodic", [False, True])
def test_tfim_local_energy_fp64(periodic):
    mc = with_batch(CONFIGS["tfim_small"], 64, periodic=periodic, gamma=0.9)
    say(f"tfim fp64 periodic={periodic}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "f64"), dev_spins(s)
    E_ref, r_ref = tfim.eloc_network_naive(mc, theta, s, return_ratios=True)
    for mode in (vq.DEDUP, vq.PLAIN):
        out = vq.local_energy(cfg, p, sp, mode, ratios=True)
        E, R = host(out["eloc"]), host(out["ratios"])
        assert np.allclose(E, E_ref, rtol=1e-10, atol=0), mode
        assert np.allclose(R[:, :mc.N], np.stack(r_ref), rtol=1e-10,
                           atol=0), mode
        assert (R[:, mc.N:] == 0).all()


def test_tfim_bf16_paper_chain_full_batch():
    mc = CONFIGS["tfim"]
    say(f"tfim bf16 N={mc.N} full batch {mc.batch}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    out = vq.local_energy(cfg, p, sp, vq.DEDUP, ratios=True)
    E, R = host(out["eloc"]), host(out["ratios"])
    P = net.unpack(mc, theta)
    rng = np.random.default_rng(12)
    picks = []
    for b in rng.choice(mc.batch, 2, replace=False):
        diag = tfim.diagonal(s[b:b + 1], mc.N, mc.periodic, mc.J)[0]
        assert abs(E[b] - (diag - mc.gamma * R[b, :mc.N].sum())) <= \
            1e-12 * max(1.0, abs(E[b]))
        picks.append((int(b), sorted(rng.choice(mc.N, 8, replace=False))))

    rel, explained = check_ratios(mc, P, cfg, p, s, R, picks, 1e-3)
    say(f"tfim bf16 ratios: max {rel.max():.2e}, {len(explained)} explained")
    small = with_batch(mc, 4)
    s4 = dev_spins(s[:4])
    ra = host(vq.local_energy(vq.make_config(small), p, s4, vq.PLAIN,
                              ratios=True)["ratios"])
    rb = host(vq.local_energy(vq.make_config(small), p, s4, vq.DEDUP,
                              ratios=True)["ratios"])
    assert np.allclose(rb, ra, rtol=1e-12, atol=0)


def test_tfim_vmc_step_fp64_equals_oracle():
    mc = with_batch(CONFIGS["tfim_small"], 32)
    say("tfim vmc step fp64")
    theta = make_params(mc)
    u = np.random.default_rng(43).random((mc.batch, mc.N))
    p = dev_params(theta, "f64")
    lr = 0.05
    out = vq.vmc_step(vq.make_config(mc), p, torch.tensor(u, device="cuda"),
                      lr)
    s_ref, _, _ = sampling.sample(mc, theta, u)
    assert np.array_equal(host(out["spins"]), s_ref)
    E = tfim.eloc_network_naive(mc, theta, s_ref)
    assert np.allclose(host(out["eloc"]), E, rtol=1e-10, atol=0)
    w = 2.0 * (E - E.mean()) / E.size
    g = ograd.grad_logpsi(mc, theta, s_ref, weights=w)
    d_gpu = host(p) - theta
    assert np.abs(d_gpu + lr * g).max() <= 1e-9 * lr * np.abs(g).max()
