"""Helpers shared by the GPU tests: device copies of seeded inputs."""
import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq

needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(),
                               reason="no GPU visible")


def dev_params(theta, precision):
    dt = torch.float64 if precision in ("f64", vq.F64) else torch.float32
    return torch.tensor(np.asarray(theta), dtype=dt, device="cuda")


def dev_spins(spins):
    return torch.tensor(np.asarray(spins, dtype=np.int8), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def say(msg):
    print(msg, flush=True)
