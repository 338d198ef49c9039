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
