"""Seeded generators: spin batches and flat parameter buffers.

Spins: each row is an independent uniformly random permutation of N/2 up and
N/2 down spins (the Sz=0 sector), int8 in {+1,-1}, drawn from
numpy.random.default_rng(cfg.spin_seed).  Duplicate rows are allowed.

Parameters: theta = 0.1 * default_rng(cfg.param_seed).standard_normal(P) over
the flat layout, then every LayerNorm gain is set to 1 and every bias to 0.
For bfloat16 workloads the values are then rounded to the nearest bfloat16
(ties to even), so the oracle and the GPU see the very same parameters.
"""
import numpy as np

from .layout import param_layout, param_count


def make_spins(cfg, batch=None, seed=None, sector_sz0=None):
    """Spins [B][N]: Sz = 0 permutations for the Heisenberg workloads,
    independent uniform +-1 for the transverse-field Ising chain (its
    Hamiltonian does not conserve Sz)."""
    if sector_sz0 is None:
        sector_sz0 = getattr(cfg, "hamiltonian", "heisenberg") != "tfim"
    return _make_spins(cfg, batch, seed, sector_sz0)


def _make_spins(cfg, batch, seed, sector_sz0):
    B = cfg.batch if batch is None else batch
    rng = np.random.default_rng(cfg.spin_seed if seed is None else seed)
    N = cfg.N
    if sector_sz0:
        base = np.array([1] * (N // 2) + [-1] * (N - N // 2), dtype=np.int8)
        out = np.empty((B, N), dtype=np.int8)
        for b in range(B):
            out[b] = rng.permutation(base)
        return out
    return np.where(rng.random((B, N)) < 0.5, 1, -1).astype(np.int8)


def bf16_round(x):
    """Nearest bfloat16 value of every entry (round half to even), float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def make_params(cfg, seed=None, std=0.1, bf16_exact=None):
    if bf16_exact is None:
        bf16_exact = cfg.precision == "bf16"
    P = param_count(cfg)
    rng = np.random.default_rng(cfg.param_seed if seed is None else seed)
    theta = std * rng.standard_normal(P)
    for name, shape, kind, off, n in param_layout(cfg):
        if kind == "gain":
            theta[off:off + n] = 1.0
        elif kind == "bias":
            theta[off:off + n] = 0.0
    if bf16_exact:
        theta = bf16_round(theta)
    return theta  # float64; callers cast to the precision they need


def scale_codebooks(cfg, theta, alpha):
    """Copy of theta with every codebook multiplied by alpha (redundancy
    sweep input: larger codebooks make the codes less sensitive)."""
    out = np.array(theta, copy=True)
    for name, shape, kind, off, n in param_layout(cfg):
        if name.endswith("codebook"):
            out[off:off + n] *= alpha
    if cfg.precision == "bf16":
        out = bf16_round(out)
    return out
