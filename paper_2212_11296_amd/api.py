"""ctypes binding of the C ABI in include/vqnqs.h (same entry-point names)."""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))

F64, F32, BF16 = 0, 1, 2
PLAIN, DEDUP = 0, 1
FLAG_CERTIFIED_VQ = 1
NCOUNTERS = 96
CTR = dict(samples=0, neighbours=1, attn_rows=2, attn_pairs=3, vq_rows=4,
           vq_certified=5, qkv_rows=6, mlp_rows=7, head_rows=8, tail_rows=9,
           changed0=16)
_PREC = {"f64": F64, "f32": F32, "bf16": BF16}
HEISENBERG_2D, TFIM_1D = 0, 1
_HAM = {"heisenberg": HEISENBERG_2D, "tfim": TFIM_1D}
_STATUS = {0: "ok", 1: "null pointer", 2: "invalid config", 3: "invalid shape",
           4: "workspace too small", 5: "unsupported configuration",
           6: "spin value other than +1/-1", 7: "HIP runtime error",
           8: "one sample's workspace exceeds the static scratch"}
STATIC_SCRATCH_BYTES = 512 << 20

WS_FORWARD, WS_GRAD, WS_SAMPLE, WS_VMC = -1, -3, -4, -5
MULTI_CONCURRENT, MULTI_GRAPH = 1, 2
EXPORTS = ["vqnqs_param_count", "vqnqs_workspace_size", "vqnqs_neighbours",
           "vqnqs_forward_logpsi", "vqnqs_local_energy", "vqnqs_grad_logpsi",
           "vqnqs_local_energy_static", "vqnqs_forward_activations",
           "vqnqs_probe_exp_rate", "vqnqs_probe_gelu", "vqnqs_sample", "vqnqs_vmc_step",
           "vqnqs_workspace_size_multi", "vqnqs_local_energy_multi",
           "vqnqs_autotune", "vqnqs_set_tuning",
           "vqnqs_workspace_status", "vqnqs_status_string",
           "vqnqs_profile_enable", "vqnqs_profile_reset", "vqnqs_profile_read"]


class VQNQSError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__(f"{fn}: {_STATUS.get(status, status)} ({status})")


class Config(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("periodic", ctypes.c_int32),
                ("marshall", ctypes.c_int32), ("J", ctypes.c_double),
                ("d_model", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("n_heads", ctypes.c_int32), ("d_ff", ctypes.c_int32),
                ("codebook_size", ctypes.c_int32), ("vq_heads", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("hamiltonian", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("attn_tail", ctypes.c_int32), ("group", ctypes.c_int32),
                ("encoder", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("cfg", Config), ("params", ctypes.c_void_p),
                ("spins", ctypes.c_void_p), ("batch", ctypes.c_int64),
                ("eloc", ctypes.c_void_p), ("stats", ctypes.c_void_p),
                ("ratios", ctypes.c_void_p), ("counters", ctypes.c_void_p)]


def n_sites(cfg):
    """Sites N of a config: L*L on the square lattice, L on the chain."""
    return cfg.L if cfg.hamiltonian == TFIM_1D else cfg.L * cfg.L


def n_tokens(cfg):
    """Sequence length: sites / spins per token."""
    return n_sites(cfg) // (cfg.group if cfg.group else 1)


def make_config(mc, precision=None, flags=0):
    """Config from any object with the workload fields (L, d_model, ...)."""
    prec = mc.precision if precision is None else precision
    prec = _PREC.get(prec, prec)
    ham = getattr(mc, "hamiltonian", "heisenberg")
    ham = _HAM.get(ham, ham)
    return Config(mc.L, int(mc.periodic), int(mc.marshall), float(mc.J),
                  mc.d_model, mc.n_layers, mc.n_heads, mc.d_ff,
                  mc.codebook_size, mc.vq_heads, int(prec), int(flags),
                  int(ham), float(getattr(mc, "gamma", 0.0)),
                  int(bool(getattr(mc, "attn_tail", False))),
                  int(getattr(mc, "group", 1)),
                  int(bool(getattr(mc, "encoder", False))))


_lib = None


def library_path():
    return os.path.join(PKG, "libvqnqs.so")


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is not built: run paper_2212_11296_amd.build.build() "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, I64, I32, SZ = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                       ctypes.c_size_t)
    C = ctypes.POINTER(Config)
    lib.vqnqs_param_count.argtypes = [C]
    lib.vqnqs_param_count.restype = I64
    lib.vqnqs_workspace_size.argtypes = [C, I64, I32, I64,
                                         ctypes.POINTER(SZ)]
    lib.vqnqs_workspace_size.restype = ctypes.c_int
    lib.vqnqs_neighbours.argtypes = [C, P, I64, P, P, P, P, SZ, P]
    lib.vqnqs_neighbours.restype = ctypes.c_int
    lib.vqnqs_forward_logpsi.argtypes = [C, P, P, I64, P, P, P, SZ, P]
    lib.vqnqs_forward_logpsi.restype = ctypes.c_int
    lib.vqnqs_forward_activations.argtypes = [C, P, P, I64, P, P, P, P, SZ,
                                              P]
    lib.vqnqs_forward_activations.restype = ctypes.c_int
    lib.vqnqs_local_energy.argtypes = [C, P, P, I64, I32, P, P, P, P, P, SZ,
                                       P]
    lib.vqnqs_local_energy.restype = ctypes.c_int
    lib.vqnqs_local_energy_static.argtypes = [C, P, P, I64, I32, P, P, P, P,
                                              P, P]
    lib.vqnqs_local_energy_static.restype = ctypes.c_int
    lib.vqnqs_sample.argtypes = [C, P, P, I64, P, P, P, SZ, P]
    lib.vqnqs_sample.restype = ctypes.c_int
    lib.vqnqs_vmc_step.argtypes = [C, P, P, I64, ctypes.c_double, P, I64, P,
                                   P, P, P, SZ, P]
    lib.vqnqs_vmc_step.restype = ctypes.c_int
    lib.vqnqs_grad_logpsi.argtypes = [C, P, P, I64, P, P, P, P, SZ, P]
    lib.vqnqs_grad_logpsi.restype = ctypes.c_int
    J = ctypes.POINTER(Job)
    lib.vqnqs_workspace_size_multi.argtypes = [J, I32, I32, ctypes.POINTER(SZ)]
    lib.vqnqs_workspace_size_multi.restype = ctypes.c_int
    lib.vqnqs_local_energy_multi.argtypes = [J, I32, I32, I32, P, SZ, P]
    lib.vqnqs_local_energy_multi.restype = ctypes.c_int
    lib.vqnqs_autotune.argtypes = [C, P, P, I64, I32, P, SZ, P,
                                   ctypes.POINTER(I32)]
    lib.vqnqs_autotune.restype = ctypes.c_int
    lib.vqnqs_set_tuning.argtypes = [C, ctypes.POINTER(I32)]
    lib.vqnqs_set_tuning.restype = ctypes.c_int
    lib.vqnqs_workspace_status.argtypes = [P, P]
    lib.vqnqs_workspace_status.restype = ctypes.c_int
    lib.vqnqs_probe_exp_rate.argtypes = [P, P, ctypes.POINTER(ctypes.c_double)]
    lib.vqnqs_probe_exp_rate.restype = ctypes.c_int
    lib.vqnqs_probe_gelu.argtypes = [P, P, ctypes.c_int64, P]
    lib.vqnqs_probe_gelu.restype = ctypes.c_int
    lib.vqnqs_status_string.argtypes = [ctypes.c_int]
    lib.vqnqs_status_string.restype = ctypes.c_char_p
    lib.vqnqs_profile_enable.argtypes = [ctypes.c_int]
    lib.vqnqs_profile_enable.restype = None
    lib.vqnqs_profile_reset.argtypes = []
    lib.vqnqs_profile_reset.restype = None
    lib.vqnqs_profile_read.argtypes = [ctypes.c_char_p, ctypes.c_int, P, P,
                                       ctypes.c_int]
    lib.vqnqs_profile_read.restype = ctypes.c_int
    _lib = lib
    return lib


def exported_symbols():
    lib = load_library()
    return {name: hasattr(lib, name) for name in EXPORTS}


def profile_enable(on=True):
    load_library().vqnqs_profile_enable(1 if on else 0)


def profile_reset():
    load_library().vqnqs_profile_reset()


def profile_read(max_kernels=64):
    """{kernel class: (total device ms, launches)} from the library's event
    timing (waits for the recorded events)."""
    lib = load_library()
    L = 48
    names = ctypes.create_string_buffer(L * max_kernels)
    ms = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_longlong * max_kernels)()
    n = lib.vqnqs_profile_read(names, L, ctypes.cast(ms, ctypes.c_void_p),
                               ctypes.cast(cnt, ctypes.c_void_p), max_kernels)
    out = {}
    for k in range(min(n, max_kernels)):
        nm = names.raw[k * L:(k + 1) * L].split(b"\0", 1)[0].decode()
        out[nm] = (ms[k], cnt[k])
    return out


def probe_exp_rate():
    """Exponentials per second the device's vector units issue."""
    import torch
    sink = torch.empty(1, dtype=torch.float32, device="cuda")
    out = ctypes.c_double(0.0)
    _check("vqnqs_probe_exp_rate", load_library().vqnqs_probe_exp_rate(
        _ptr(sink), _stream(), ctypes.byref(out)))
    return out.value


def probe_gelu(x):
    """GELU of a device float32 tensor by the BF16 MLP's device function."""
    import torch
    y = torch.empty_like(x)
    _check("vqnqs_probe_gelu", load_library().vqnqs_probe_gelu(
        _ptr(x), _ptr(y), x.numel(), _stream()))
    return y


def _check(fn, st):
    if st != 0:
        raise VQNQSError(fn, st)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def param_count(cfg):
    n = load_library().vqnqs_param_count(ctypes.byref(cfg))
    if n < 0:
        raise VQNQSError("vqnqs_param_count", -n)
    return n


def workspace_size(cfg, batch, mode, chunk=0):
    out = ctypes.c_size_t(0)
    _check("vqnqs_workspace_size",
           load_library().vqnqs_workspace_size(ctypes.byref(cfg), batch, mode,
                                               chunk, ctypes.byref(out)))
    return out.value


def _workspace(cfg, batch, mode, ws, budget):
    import torch
    if ws is not None:
        return ws
    need_all = workspace_size(cfg, max(batch, 1), mode, 0)
    size = min(need_all, max(budget, workspace_size(cfg, max(batch, 1), mode,
                                                    1)))
    return torch.empty(size, dtype=torch.uint8, device="cuda")


def _check_status(ws):
    _check("vqnqs_workspace_status",
           load_library().vqnqs_workspace_status(_ptr(ws), _stream()))


def neighbours(cfg, spins, ws=None, check=True):
    import torch
    B = spins.shape[0]
    N = n_sites(cfg)
    ws = _workspace(cfg, B, -1, ws, 1 << 20)
    bonds = torch.empty((B, 2 * N), dtype=torch.int16, device="cuda")
    count = torch.empty(B, dtype=torch.int32, device="cuda")
    diag = torch.empty(B, dtype=torch.float64, device="cuda")
    _check("vqnqs_neighbours", load_library().vqnqs_neighbours(
        ctypes.byref(cfg), _ptr(spins), B, _ptr(bonds), _ptr(count),
        _ptr(diag), _ptr(ws), ws.numel(), _stream()))
    if check:
        _check_status(ws)
    return bonds, count, diag


def forward_logpsi(cfg, params, spins, codes=False, ws=None,
                   budget=8 << 30, check=True):
    import torch
    B = spins.shape[0]
    N = n_sites(cfg)
    ws = _workspace(cfg, B, -1, ws, budget)
    lp = torch.empty(B, dtype=torch.float64, device="cuda")
    cd = (torch.empty((B, cfg.n_layers, N, cfg.vq_heads), dtype=torch.int32,
                      device="cuda") if codes else None)
    _check("vqnqs_forward_logpsi", load_library().vqnqs_forward_logpsi(
        ctypes.byref(cfg), _ptr(params), _ptr(spins), B, _ptr(lp), _ptr(cd),
        _ptr(ws), ws.numel(), _stream()))
    if check:
        _check_status(ws)
    return (lp, cd) if codes else lp


def forward_activations(cfg, params, spins, ws=None, budget=8 << 30,
                        check=True):
    """log psi [B], codes [B][n_layers][T][H] and every layer's attention
    output [B][n_layers][T][d] (float64 in the F64 mode, else float32); T
    token positions (the sites with one spin per token)."""
    import torch
    B = spins.shape[0]
    N = n_tokens(cfg)
    ws = _workspace(cfg, B, -1, ws, budget)
    lp = torch.empty(B, dtype=torch.float64, device="cuda")
    cd = torch.empty((B, cfg.n_layers, N, cfg.vq_heads), dtype=torch.int32,
                     device="cuda")
    at = torch.empty((B, cfg.n_layers, N, cfg.d_model),
                     dtype=torch.float64 if cfg.precision == F64
                     else torch.float32, device="cuda")
    _check("vqnqs_forward_activations",
           load_library().vqnqs_forward_activations(
               ctypes.byref(cfg), _ptr(params), _ptr(spins), B, _ptr(lp),
               _ptr(cd), _ptr(at), _ptr(ws), ws.numel(), _stream()))
    if check:
        _check_status(ws)
    return lp, cd, at


def local_energy(cfg, params, spins, mode=DEDUP, stats=True, ratios=False,
                 counters=False, ws=None, budget=8 << 30, check=True,
                 out=None):
    """Returns a dict of device tensors: eloc [B], and optionally stats [2]
    (mean, variance), ratios [B][2N], counters [NCOUNTERS]."""
    import torch
    B = spins.shape[0]
    N = n_sites(cfg)
    ws = _workspace(cfg, B, mode, ws, budget)
    o = out if out is not None else {}
    if "eloc" not in o:
        o["eloc"] = torch.empty(B, dtype=torch.float64, device="cuda")
    if stats and "stats" not in o:
        o["stats"] = torch.empty(2, dtype=torch.float64, device="cuda")
    if ratios and "ratios" not in o:
        o["ratios"] = torch.empty((B, 2 * N), dtype=torch.float64,
                                  device="cuda")
    if counters and "counters" not in o:
        o["counters"] = torch.empty(NCOUNTERS, dtype=torch.int64,
                                    device="cuda")
    _check("vqnqs_local_energy", load_library().vqnqs_local_energy(
        ctypes.byref(cfg), _ptr(params), _ptr(spins), B, mode,
        _ptr(o["eloc"]), _ptr(o.get("stats")), _ptr(o.get("ratios")),
        _ptr(o.get("counters")), _ptr(ws), ws.numel(), _stream()))
    if check:
        _check_status(ws)
    return o


def local_energy_static(cfg, params, spins, mode=DEDUP, stats=True,
                        ratios=False, counters=False, check=True, out=None):
    """vqnqs_local_energy_static: the local energy in the library's own
    static device array (no workspace argument, nothing allocated by the
    call).  Same outputs as local_energy plus "status" [1] int32, the call's
    status word."""
    import torch
    B = spins.shape[0]
    N = n_sites(cfg)
    o = out if out is not None else {}
    if "eloc" not in o:
        o["eloc"] = torch.empty(B, dtype=torch.float64, device="cuda")
    if stats and "stats" not in o:
        o["stats"] = torch.empty(2, dtype=torch.float64, device="cuda")
    if ratios and "ratios" not in o:
        o["ratios"] = torch.empty((B, 2 * N), dtype=torch.float64,
                                  device="cuda")
    if counters and "counters" not in o:
        o["counters"] = torch.empty(NCOUNTERS, dtype=torch.int64,
                                    device="cuda")
    if "status" not in o:
        o["status"] = torch.empty(1, dtype=torch.int32, device="cuda")
    _check("vqnqs_local_energy_static",
           load_library().vqnqs_local_energy_static(
               ctypes.byref(cfg), _ptr(params), _ptr(spins), B, mode,
               _ptr(o["eloc"]), _ptr(o.get("stats")), _ptr(o.get("ratios")),
               _ptr(o.get("counters")), _ptr(o["status"]), _stream()))
    if check:
        _check("vqnqs_local_energy_static", int(o["status"].item()))
    return o


def sample(cfg, params, uniforms, ws=None, budget=8 << 30, check=True,
           out=None):
    """Direct samples s ~ psi^2 (chain rule) drawn with the caller's
    uniform numbers (device float64 [B][N]); returns (spins int8 [B][N],
    log psi float64 [B])."""
    import torch
    B, N = uniforms.shape
    assert N == n_sites(cfg) and uniforms.dtype == torch.float64
    ws = _workspace(cfg, B, WS_SAMPLE, ws, budget)
    o = out if out is not None else {}
    if "spins" not in o:
        o["spins"] = torch.empty((B, N), dtype=torch.int8, device="cuda")
    if "logpsi" not in o:
        o["logpsi"] = torch.empty(B, dtype=torch.float64, device="cuda")
    u = uniforms.contiguous()
    _check("vqnqs_sample", load_library().vqnqs_sample(
        ctypes.byref(cfg), _ptr(params), _ptr(u), B, _ptr(o["spins"]),
        _ptr(o["logpsi"]), _ptr(ws), ws.numel(), _stream()))
    if check:
        _check_status(ws)
    return o["spins"], o["logpsi"]


def vmc_step(cfg, params, uniforms, lr, opt_state=None, step=1, ws=None,
             budget=8 << 30, check=True, out=None):
    """One VMC step on the device (sample, local energy, energy gradient,
    update of ``params`` in place).  opt_state: None for gradient descent,
    else a zeroed device tensor [2][P] of the parameters' dtype (Adam).
    Returns a dict with spins [B][N], eloc [B] and stats [2] of the step."""
    import torch
    B, N = uniforms.shape
    assert N == n_sites(cfg) and uniforms.dtype == torch.float64
    if ws is None:
        need = workspace_size(cfg, B, WS_VMC, 0)
        if need > budget:
            c = 1
            while (c * 2 <= B
                   and workspace_size(cfg, B, WS_VMC, c * 2) <= budget):
                c *= 2
            need = workspace_size(cfg, B, WS_VMC, c)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    o = out if out is not None else {}
    if "spins" not in o:
        o["spins"] = torch.empty((B, N), dtype=torch.int8, device="cuda")
    if "eloc" not in o:
        o["eloc"] = torch.empty(B, dtype=torch.float64, device="cuda")
    if "stats" not in o:
        o["stats"] = torch.empty(2, dtype=torch.float64, device="cuda")
    _check("vqnqs_vmc_step", load_library().vqnqs_vmc_step(
        ctypes.byref(cfg), _ptr(params), _ptr(opt_state), int(step),
        float(lr), _ptr(uniforms.contiguous()), B, _ptr(o["spins"]),
        _ptr(o["eloc"]), _ptr(o["stats"]), _ptr(ws), ws.numel(), _stream()))
    if check:
        _check_status(ws)
    return o


def grad_logpsi(cfg, params, spins, weights=None, logpsi=False, ws=None,
                budget=8 << 30, check=True, out=None):
    """Straight-through gradient of log psi (device tensor, params' dtype):
    [P] weighted by ``weights`` (device float64 [B]) if given, else [B][P]."""
    import torch
    B = spins.shape[0]
    P = param_count(cfg)
    ws = _workspace(cfg, B, WS_GRAD, ws, budget)
    shape = (P,) if weights is not None else (B, P)
    g = (out if out is not None
         else torch.empty(shape, dtype=params.dtype, device="cuda"))
    lp = torch.empty(B, dtype=torch.float64, device="cuda") if logpsi else None
    w = None
    if weights is not None:
        w = weights.to(device="cuda", dtype=torch.float64).contiguous()
        if w.numel() == 0:
            # an empty tensor has no address; the weighted form is selected
            # by a non-NULL pointer
            w = torch.zeros(1, dtype=torch.float64, device="cuda")
    _check("vqnqs_grad_logpsi", load_library().vqnqs_grad_logpsi(
        ctypes.byref(cfg), _ptr(params), _ptr(spins), B, _ptr(w), _ptr(g),
        _ptr(lp), _ptr(ws), ws.numel(), _stream()))
    if check:
        _check_status(ws)
    return (g, lp) if logpsi else g


def _logpsi_function():
    import torch

    class LogPsi(torch.autograd.Function):
        """log psi(spins) as a differentiable function of the parameters:
        forward by vqnqs_forward_logpsi, backward by vqnqs_grad_logpsi with
        the incoming gradient as the sample weights."""

        @staticmethod
        def forward(ctx, params, spins, cfg):
            ctx.save_for_backward(params, spins)
            ctx.cfg = cfg
            return forward_logpsi(cfg, params, spins)

        @staticmethod
        def backward(ctx, grad_out):
            params, spins = ctx.saved_tensors
            g = grad_logpsi(ctx.cfg, params, spins, weights=grad_out)
            return g, None, None

    return LogPsi


def logpsi(cfg, params, spins):
    """Differentiable log psi [B] (autograd through the HIP backward)."""
    return _logpsi_function().apply(params, spins, cfg)


def _jobs_array(jobs, outs):
    arr = (Job * len(jobs))()
    for i, ((cfg, params, spins), o) in enumerate(zip(jobs, outs)):
        arr[i].cfg = cfg
        arr[i].params = params.data_ptr()
        arr[i].spins = spins.data_ptr()
        arr[i].batch = spins.shape[0]
        arr[i].eloc = o["eloc"].data_ptr()
        arr[i].stats = o["stats"].data_ptr() if "stats" in o else None
        arr[i].ratios = o["ratios"].data_ptr() if "ratios" in o else None
        arr[i].counters = (o["counters"].data_ptr() if "counters" in o
                           else None)
    return arr


def workspace_size_multi(jobs, mode=DEDUP):
    """jobs: list of (cfg, params, spins)."""
    out = ctypes.c_size_t(0)
    arr = (Job * len(jobs))()
    for i, (cfg, params, spins) in enumerate(jobs):
        arr[i].cfg = cfg
        arr[i].batch = spins.shape[0]
    _check("vqnqs_workspace_size_multi", load_library().vqnqs_workspace_size_multi(
        arr, len(jobs), mode, ctypes.byref(out)))
    return out.value


def local_energy_multi(jobs, mode=DEDUP, flags=MULTI_CONCURRENT | MULTI_GRAPH,
                       ws=None, budget=8 << 30, ratios=False, stats=True,
                       outs=None, check=True):
    """Local energies of several lattices in one call.  jobs: list of
    (cfg, params, spins).  Returns one dict of device outputs per job; pass
    the same ``outs`` (and ``ws``) back to replay the captured graph."""
    import torch
    if outs is None:
        outs = []
        for cfg, params, spins in jobs:
            B, N = spins.shape[0], n_sites(cfg)
            o = {"eloc": torch.empty(B, dtype=torch.float64, device="cuda")}
            if stats:
                o["stats"] = torch.empty(2, dtype=torch.float64, device="cuda")
            if ratios:
                o["ratios"] = torch.empty((B, 2 * N), dtype=torch.float64,
                                          device="cuda")
            outs.append(o)
    if ws is None:
        need = workspace_size_multi(jobs, mode)
        ws = torch.empty(min(need, budget), dtype=torch.uint8, device="cuda")
    arr = _jobs_array(jobs, outs)
    _check("vqnqs_local_energy_multi", load_library().vqnqs_local_energy_multi(
        arr, len(jobs), mode, flags, _ptr(ws), ws.numel(), _stream()))
    if check:
        _check_status(ws)      # the OR of every job's status word
    return outs


def autotune(cfg, params, spins, mode=DEDUP, ws=None, budget=8 << 30):
    """Times the matrix-core launch variants on these samples and keeps the
    fastest for this model width; returns the choices [qkv, mlp, vq]."""
    import torch
    B = spins.shape[0]
    if ws is None:
        need = workspace_size(cfg, max(B, 1), mode, 0) + 8 * B + 256
        ws = torch.empty(min(need, budget + 8 * B + 256), dtype=torch.uint8,
                         device="cuda")
    ch = (ctypes.c_int32 * 3)()
    _check("vqnqs_autotune", load_library().vqnqs_autotune(
        ctypes.byref(cfg), _ptr(params), _ptr(spins), B, mode, _ptr(ws),
        ws.numel(), _stream(), ch))
    return list(ch)


def set_tuning(cfg, choices):
    ch = (ctypes.c_int32 * 3)(*choices)
    _check("vqnqs_set_tuning",
           load_library().vqnqs_set_tuning(ctypes.byref(cfg), ch))
