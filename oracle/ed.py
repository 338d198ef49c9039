"""Exact diagonalisation of the 2-D Heisenberg model (paper Sec. 4).

The Hamiltonian is built from Pauli matrices and Kronecker products, with no
use of the spin-exchange enumeration in ``lattice``:

    H = J * sum_<ij> (X_i X_j + Y_i Y_j + Z_i Z_j) / 4      (S = sigma / 2)

Basis: site 0 is the most significant tensor factor; spin +1 is |0> (Z = +1)
and spin -1 is |1>, so a configuration s has index sum_i [s_i = -1] 2^(N-1-i).
The Marshall rotation multiplies basis state s by (-1)^(number of up spins
on sublattice B), B = sites with r + c odd.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import eigsh

from .lattice import bonds

_X = sp.csr_matrix(np.array([[0, 1], [1, 0]], dtype=np.complex128))
_Y = sp.csr_matrix(np.array([[0, -1j], [1j, 0]], dtype=np.complex128))
_Z = sp.csr_matrix(np.array([[1, 0], [0, -1]], dtype=np.complex128))


def _site_op(op, i, N):
    left = sp.identity(2 ** i, dtype=np.complex128, format="csr")
    right = sp.identity(2 ** (N - 1 - i), dtype=np.complex128, format="csr")
    return sp.kron(sp.kron(left, op, format="csr"), right, format="csr")


def hamiltonian(L, periodic=True, J=1.0, marshall=True):
    """Real sparse H on the full 2^N space (optionally Marshall-rotated)."""
    N = L * L
    ops = {}
    for name, op in (("x", _X), ("y", _Y), ("z", _Z)):
        ops[name] = [_site_op(op, i, N) for i in range(N)]
    H = sp.csr_matrix((2 ** N, 2 ** N), dtype=np.complex128)
    for _, i, j in bonds(L, periodic):
        H = H + (ops["x"][i] @ ops["x"][j] + ops["y"][i] @ ops["y"][j]
                 + ops["z"][i] @ ops["z"][j]) * (0.25 * J)
    if abs(H.imag).max() > 0:
        raise AssertionError("Heisenberg Hamiltonian must be real")
    H = H.real.tocsr()
    if marshall:
        sgn = marshall_signs(L)
        D = sp.diags(sgn)
        H = (D @ H @ D).tocsr()
    return H


def config_of_index(idx, N):
    """Spin configuration(s) [.., N] of basis index/indices."""
    idx = np.asarray(idx, dtype=np.int64)
    bits = (idx[..., None] >> (N - 1 - np.arange(N))) & 1
    return np.where(bits == 1, -1, 1).astype(np.int8)


def index_of_config(spins):
    s = np.atleast_2d(spins)
    N = s.shape[1]
    w = (1 << (N - 1 - np.arange(N))).astype(np.int64)
    return ((s < 0).astype(np.int64) * w).sum(axis=1)


def marshall_signs(L):
    N = L * L
    idx = np.arange(2 ** N, dtype=np.int64)
    s = config_of_index(idx, N)
    sub_b = np.array([(r + c) % 2 == 1 for r in range(L) for c in range(L)])
    n_up_b = ((s == 1) & sub_b[None, :]).sum(axis=1)
    return np.where(n_up_b % 2 == 0, 1.0, -1.0)


def sz0_indices(N):
    idx = np.arange(2 ** N, dtype=np.int64)
    pop = np.zeros(2 ** N, dtype=np.int64)
    for bit in range(N):
        pop += (idx >> bit) & 1
    return idx[pop == N // 2]


def ground_state(L, periodic=True, J=1.0, marshall=True):
    """(E0, sector indices, ground-state vector on the Sz=0 sector)."""
    H = hamiltonian(L, periodic, J, marshall)
    sec = sz0_indices(L * L)
    Hs = H[sec][:, sec]
    vals, vecs = eigsh(Hs, k=1, which="SA", tol=1e-12)
    v = vecs[:, 0]
    if v.sum() < 0:
        v = -v
    return float(vals[0]), sec, v, Hs
