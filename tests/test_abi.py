"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/vqnqs.h, counts parameters like the workload layout, and
rejects bad arguments on the host before any HIP call."""
import ctypes
from dataclasses import replace
import os
import re
import subprocess

import pytest

import paper_2212_11296_amd as vq
from workloads import CONFIGS, MULTI_LATTICE, param_count

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "vqnqs.h")).read()
    return sorted(set(re.findall(r"\b(vqnqs_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = vq.load_library()
    declared = header_functions()
    assert len(declared) >= 7
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", vq.library_path()],
                         capture_output=True, text=True).stdout
    for name in declared:
        assert re.search(rf"\bT {name}$", out, re.M), name


@pytest.mark.parametrize("mc", list(CONFIGS.values()) + list(MULTI_LATTICE))
def test_param_count_matches_layout(mc):
    assert vq.param_count(vq.make_config(mc)) == param_count(mc)


def _cfg(**kw):
    c = vq.make_config(CONFIGS["small"])
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw,status", [
    (dict(L=2), 2),                       # periodic needs L >= 3
    (dict(L=5), 2),                       # periodic + Marshall needs even L
    (dict(d_model=17), 2),                # d % n_heads
    (dict(d_model=18), 5),                # head width 9 unsupported
    (dict(vq_heads=3), 2),                # d % vq_heads
    (dict(precision=7), 2),
    (dict(flags=4), 2),
    (dict(n_heads=16), 5),                # head width 1 unsupported
    (dict(codebook_size=0), 2),
    (dict(hamiltonian=1), 2),             # chain with the Marshall flag
    (dict(hamiltonian=1, marshall=0, L=1025), 2),   # chain longer than 1024
    (dict(hamiltonian=1, marshall=0, L=2), 2),      # periodic chain of 2
    (dict(hamiltonian=1, marshall=0, gamma=float("nan")), 2),
    (dict(hamiltonian=5), 2),
    (dict(group=5), 2),                   # at most 4 spins per token
    (dict(group=3), 2),                   # 16 sites in tokens of 3
    (dict(group=-1), 2),
    (dict(encoder=2), 2),
    (dict(encoder=1, attn_tail=1), 2),    # the half-block is a decoder's
    (dict(encoder=1, flags=2), 5),        # no rank-|C| attention update
])
def test_invalid_configs_rejected(kw, status):
    lib = vq.load_library()
    c = _cfg(**kw)
    assert lib.vqnqs_param_count(ctypes.byref(c)) == -status
    sz = ctypes.c_size_t()
    assert lib.vqnqs_workspace_size(ctypes.byref(c), 4, 1, 0,
                                    ctypes.byref(sz)) == status
    assert lib.vqnqs_local_energy(ctypes.byref(c), None, None, 4, 1, None,
                                  None, None, None, None, 0, None) == status


@pytest.mark.parametrize("group", [1, 4])
def test_encoder_param_count_matches_layout(group):
    mc = replace(CONFIGS["small"], name="small_enc", encoder=True, group=group)
    assert vq.param_count(vq.make_config(mc)) == param_count(mc)
    dec = replace(mc, encoder=False)
    # one token row fewer (no beginning of sequence) and one head output
    V = 1 << group
    assert param_count(dec) - param_count(mc) == mc.d_model + (V - 1) * (mc.d_model + 1)


def test_gelu_probe_host_errors():
    lib = vq.load_library()
    assert lib.vqnqs_probe_gelu(None, None, 0, None) == 0
    assert lib.vqnqs_probe_gelu(None, None, -1, None) == 3
    assert lib.vqnqs_probe_gelu(None, None, 4, None) == 1


def test_open_odd_lattice_allowed():
    c = _cfg(L=5, periodic=0)
    assert vq.param_count(c) > 0


def test_null_and_shape_errors_on_host():
    lib = vq.load_library()
    c = _cfg()
    dummy = ctypes.c_void_p(16)           # never dereferenced: errors first
    assert lib.vqnqs_local_energy(None, dummy, dummy, 4, 1, dummy, None, None,
                                  None, dummy, 1 << 20, None) == 1
    assert lib.vqnqs_local_energy(ctypes.byref(c), dummy, dummy, -1, 1, dummy,
                                  None, None, None, dummy, 1 << 20, None) == 3
    assert lib.vqnqs_local_energy(ctypes.byref(c), None, dummy, 4, 1, dummy,
                                  None, None, None, dummy, 1 << 20, None) == 1
    assert lib.vqnqs_local_energy(ctypes.byref(c), dummy, dummy, 4, 9, dummy,
                                  None, None, None, dummy, 1 << 20, None) == 2
    assert lib.vqnqs_forward_logpsi(ctypes.byref(c), dummy, dummy, 4, None,
                                    None, dummy, 1 << 20, None) == 1
    assert lib.vqnqs_neighbours(ctypes.byref(c), dummy, -2, dummy, dummy,
                                None, dummy, 1 << 20, None) == 3
    assert lib.vqnqs_workspace_status(None, None) == 1
    assert lib.vqnqs_status_string(6) == b"spin value other than +1/-1"


def test_workspace_size_grows_with_chunk():
    for name in ["small", "medium", "large"]:
        c = vq.make_config(CONFIGS[name])
        for mode in (vq.PLAIN, vq.DEDUP, -1):
            s1 = vq.workspace_size(c, 64, mode, 1)
            s8 = vq.workspace_size(c, 64, mode, 8)
            sall = vq.workspace_size(c, 64, mode, 0)
            assert 0 < s1 < s8 < sall


def test_gradient_multi_and_tuning_errors_on_host():
    """Argument errors of the gradient, multi-lattice and tuning entry points
    are detected on the host, before any HIP call."""
    lib = vq.load_library()
    c = _cfg()
    dummy = ctypes.c_void_p(16)           # never dereferenced: errors first
    ws = 1 << 20
    # gradient: null grad, negative batch, null params
    assert lib.vqnqs_grad_logpsi(ctypes.byref(c), dummy, dummy, 4, None, None,
                                 None, dummy, ws, None) == 1
    assert lib.vqnqs_grad_logpsi(ctypes.byref(c), dummy, dummy, -1, None, dummy,
                                 None, dummy, ws, None) == 3
    assert lib.vqnqs_grad_logpsi(ctypes.byref(c), None, dummy, 4, None, dummy,
                                 None, dummy, ws, None) == 1
    bad = _cfg(d_model=17)
    assert lib.vqnqs_grad_logpsi(ctypes.byref(bad), dummy, dummy, 4, None,
                                 dummy, None, dummy, ws, None) == 2
    # multi-lattice: no jobs, too many jobs, bad mode, bad flags, null eloc
    jobs = (vq.api.Job * 2)()
    for j in jobs:
        j.cfg = c
        j.params = 16
        j.spins = 16
        j.batch = 4
        j.eloc = 16
    assert lib.vqnqs_local_energy_multi(jobs, 0, 1, 0, dummy, ws, None) == 3
    assert lib.vqnqs_local_energy_multi(jobs, 65, 1, 0, dummy, ws, None) == 3
    assert lib.vqnqs_local_energy_multi(jobs, 2, 7, 0, dummy, ws, None) == 2
    assert lib.vqnqs_local_energy_multi(jobs, 2, 1, 8, dummy, ws, None) == 2
    assert lib.vqnqs_local_energy_multi(jobs, 2, 1, 0, None, ws, None) == 1
    jobs[1].eloc = None
    assert lib.vqnqs_local_energy_multi(jobs, 2, 1, 0, dummy, ws, None) == 1
    jobs[1].eloc = 16
    jobs[0].batch = -1
    assert lib.vqnqs_local_energy_multi(jobs, 2, 1, 0, dummy, ws, None) == 3
    jobs[0].batch = 4
    jobs[0].cfg = bad
    assert lib.vqnqs_local_energy_multi(jobs, 2, 1, 0, dummy, ws, None) == 2
    # a workspace that cannot hold every job's minimum
    jobs[0].cfg = c
    assert lib.vqnqs_local_energy_multi(jobs, 2, 1, 0, dummy, 1024, None) == 4
    # tuning: choices the width does not allow, null choices
    ch = (ctypes.c_int32 * 3)(3, 1, 1)
    assert lib.vqnqs_set_tuning(ctypes.byref(c), ch) == 2
    assert lib.vqnqs_set_tuning(ctypes.byref(c), None) == 1
    large = vq.make_config(CONFIGS["large"])
    assert lib.vqnqs_set_tuning(ctypes.byref(large),
                                (ctypes.c_int32 * 3)(2, 1, 4)) == 0
    assert lib.vqnqs_set_tuning(ctypes.byref(large),
                                (ctypes.c_int32 * 3)(2, 2, 2)) == 0
    assert lib.vqnqs_autotune(ctypes.byref(c), dummy, dummy, 4, 5, dummy, ws,
                              None, None) == 2


def test_gradient_and_multi_workspace_sizes():
    for name in ["small", "medium", "grad"]:
        c = vq.make_config(CONFIGS[name])
        s1 = vq.workspace_size(c, 16, vq.WS_GRAD, 1)
        s4 = vq.workspace_size(c, 16, vq.WS_GRAD, 4)
        assert 0 < s1 < s4
        # per-sample gradients of a chunk are held in the workspace
        assert s4 - s1 >= 3 * vq.param_count(c) * (8 if name == "small" else 4)
    jobs = [(vq.make_config(m), _Shape(m.batch), _Shape(m.batch))
            for m in (CONFIGS["small"], CONFIGS["medium"])]
    total = vq.workspace_size_multi(jobs)
    parts = sum(vq.workspace_size(cfg, s.shape[0], vq.DEDUP, 0)
                for cfg, s, _ in jobs)
    assert parts <= total <= parts + 256 * (len(jobs) + 1)


class _Shape:
    """Stand-in with only a shape, for workspace queries."""
    def __init__(self, b):
        self.shape = (b,)
