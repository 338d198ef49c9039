"""One variational Monte Carlo step on the GPU (vqnqs_vmc_step: direct
samples, local energies, the energy gradient of eq. 3, the update) against
the FP64 oracle (oracle/vmc.py), through the C ABI.

* FP64 4x4, gradient descent: with the same uniform numbers the step draws
  the oracle's samples exactly, their local energies within 1e-10 and the
  parameter update within 1e-9 of its largest entry.
* FP64 4x4, Adam: the update equals Adam (b1 = 0.9, b2 = 0.999,
  eps = 1e-8, bias-corrected) applied to the oracle's gradient, within
  1e-9 on every entry whose gradient is not at the rounding level (Adam's
  first step divides a gradient by its own magnitude, so an entry of size
  1e-15 has no defined sign).
"""
import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq
from oracle import vmc
from workloads import CONFIGS, make_params, with_batch

from gpu_common import dev_params, host, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def _setup(B=64, seed=41):
    mc = with_batch(CONFIGS["small"], B)
    theta = make_params(mc)
    u = np.random.default_rng(seed).random((B, mc.N))
    return mc, theta, u


def test_vmc_step_sgd_fp64_equals_oracle():
    mc, theta, u = _setup()
    say("vmc step sgd fp64 4x4")
    lr = 0.05
    p = dev_params(theta, "f64")
    out = vq.vmc_step(vq.make_config(mc), p, torch.tensor(u, device="cuda"),
                      lr)
    new_ref, s_ref, E_ref = vmc.vmc_step_sgd(mc, theta, u, lr)
    assert np.array_equal(host(out["spins"]), s_ref)
    assert np.allclose(host(out["eloc"]), E_ref, rtol=1e-10, atol=0)
    st = host(out["stats"])
    assert abs(st[0] - E_ref.mean()) <= 1e-10 * abs(E_ref.mean())
    d_gpu = host(p) - theta
    d_ref = new_ref - theta
    assert np.abs(d_gpu - d_ref).max() <= 1e-9 * np.abs(d_ref).max()


def test_vmc_step_adam_fp64_equals_oracle():
    mc, theta, u = _setup(seed=42)
    say("vmc step adam fp64 4x4")
    lr = 0.01
    p = dev_params(theta, "f64")
    P = p.numel()
    opt = torch.zeros(2 * P, dtype=torch.float64, device="cuda")
    uu = torch.tensor(u, device="cuda")
    vq.vmc_step(vq.make_config(mc), p, uu, lr, opt_state=opt, step=1)
    th1 = host(p).copy()
    # reference: Adam on the oracle's gradient, step 1 from zero moments
    g, _ = vmc.energy_gradient_samples(
        mc, theta, vmc.sampling.sample(mc, theta, u)[0])
    m = 0.1 * g
    v = 0.001 * g * g
    ref = theta - lr * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    ok = np.abs(g) > 1e-10 * np.abs(g).max()
    assert np.abs(th1 - ref)[ok].max() <= 1e-9 * lr
    mo = host(opt)
    assert np.allclose(mo[:P][ok], m[ok], rtol=1e-9, atol=0)
    assert np.allclose(mo[P:][ok], v[ok], rtol=1e-9, atol=0)


def test_vmc_converges_on_the_4x4_heisenberg_lattice():
    """Energy optimisation end to end on the device: a 2-layer model (d=32,
    4 heads, MLP 128, 64 codes) trained by vqnqs_vmc_step with Adam from the
    seeded initialisation on the periodic 4x4 Heisenberg lattice reaches
    the exact ground-state energy (Lanczos on the Pauli-matrix Hamiltonian)
    within 3% (observed 2.3% after 1000 steps; the first steps sit 9-17%
    above it), and its energy variance falls by more than 40%."""
    from dataclasses import replace
    from oracle import ed
    mc = replace(CONFIGS["small"], precision="f32", d_model=32, n_heads=4,
                 d_ff=128, codebook_size=64, n_layers=2)
    E0 = ed.ground_state(4, periodic=True)[0]
    cfg = vq.make_config(mc)
    p = dev_params(make_params(mc), "f32")
    opt = torch.zeros(2 * p.numel(), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(1)
    B, steps = 1024, 1000
    ws = torch.empty(vq.workspace_size(cfg, B, vq.WS_VMC, 0),
                     dtype=torch.uint8, device="cuda")
    hist = torch.empty((steps, 2), dtype=torch.float64, device="cuda")
    out = None
    say("vmc 4x4, 1000 Adam steps")
    for k in range(1, steps + 1):
        u = torch.rand((B, mc.N), dtype=torch.float64, device="cuda",
                       generator=gen)
        out = vq.vmc_step(cfg, p, u, 2e-3 * 0.1 ** (k / 2000), opt_state=opt,
                          step=k, ws=ws, check=(k == 1), out=out)
        hist[k - 1] = out["stats"]
    h = host(hist)
    first, last = h[:100], h[-100:]
    rel = (last[:, 0].mean() - E0) / abs(E0)
    say(f"E0 {E0:.5f}; first 100 steps {first[:, 0].mean():.4f}, last 100 "
        f"{last[:, 0].mean():.4f} (rel {rel:.4f}); variance "
        f"{first[:, 1].mean():.3f} -> {last[:, 1].mean():.3f}")
    assert last[:, 0].mean() >= E0 - 0.05 * abs(E0)   # variational, noisy
    assert rel < 0.03
    assert last[:, 1].mean() < 0.6 * first[:, 1].mean()
