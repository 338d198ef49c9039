"""The GELU of the BF16 mode's matrix-core MLP (erf from Abramowitz &
Stegun 7.1.26, folded into one branch-free expression) against the exact
form x Phi(x) = x erfc(-x / sqrt 2) / 2 in FP64, through the C ABI.

The method's bound: |erf error| <= 1.5e-7, so |Phi error| <= 0.75e-7 and
|GELU error| <= 0.75e-7 |x|, plus the FP32 evaluation's own rounding (a few
units in the last place of terms of size |x|, below 6e-7 |x| together).
Inputs: a dense grid over [-12, 12], the integers, the values where the
expression switches between its branches (0, the signed zeros), tiny and
large magnitudes.  Negative large inputs must give a negligible magnitude
(GELU(-x) tends to 0), positive large ones x itself.
"""
import math

import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq

from gpu_common import needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def gelu_exact(x):
    x = np.asarray(x, dtype=np.float64)
    return x * np.array([0.5 * math.erfc(-v / math.sqrt(2.0)) for v in x.ravel()]
                        ).reshape(x.shape)


def test_gelu_probe_within_method_bound():
    grid = np.linspace(-12.0, 12.0, 200001, dtype=np.float32)
    special = np.array([0.0, -0.0, 1e-30, -1e-30, 1e-6, -1e-6, 0.5, -0.5,
                        1.0, -1.0, 3.0, -3.0, 30.0, -30.0, 1e4, -1e4],
                       dtype=np.float32)
    x = np.concatenate([grid, np.arange(-12, 13, dtype=np.float32), special])
    y = vq.probe_gelu(torch.tensor(x, device="cuda")).cpu().numpy()
    ref = gelu_exact(x)
    ax = np.abs(x.astype(np.float64))
    err = np.abs(y.astype(np.float64) - ref)
    bound = 0.75e-7 * ax + 6e-7 * ax + 1e-38
    worst = np.argmax(err / bound)
    say(f"gelu: max abs err {err.max():.3e}, worst ratio to bound "
        f"{(err / bound)[worst]:.3f} at x={x[worst]}")
    assert (err <= bound).all()
    assert y[x == 0.0].tolist() == [0.0] * int((x == 0.0).sum())
    assert y[x == 1e4][0] == np.float32(1e4)
    assert abs(y[x == -1e4][0]) < 1e-30


def test_gelu_probe_empty_and_errors():
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    assert vq.probe_gelu(e).numel() == 0
    lib = vq.load_library()
    assert lib.vqnqs_probe_gelu(None, None, -1, None) == 3
    assert lib.vqnqs_probe_gelu(None, None, 4, None) == 1
