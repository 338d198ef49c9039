"""One-dimensional transverse-field Ising model, FP64 (paper Sec. 4):

    H = -J sum_<ij> Z_i Z_j - Gamma sum_i X_i     (Pauli matrices)

on a chain of N sites, nearest neighbours (i, i+1), plus (N-1, 0) when
periodic (the paper's chain is open).  In the Z basis a row s of H has the
diagonal -J sum_<ij> s_i s_j and, for every site i, the configuration with
spin i flipped (k-local rows with k = 1, Sec. 2) with element -Gamma.  For
Gamma > 0 every off-diagonal element is non-positive, so the ground state
is positive and psi needs no phase.  The local energy of eq. (2) is

    E_loc(s) = -J sum_<ij> s_i s_j - Gamma sum_i psi(s^(i)) / psi(s).

``hamiltonian`` builds H from Pauli Kronecker products, independently of
the flip enumeration used by ``eloc_naive``.
"""
import itertools

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import eigsh

from . import network as net

_X = sp.csr_matrix(np.array([[0.0, 1.0], [1.0, 0.0]]))
_Z = sp.csr_matrix(np.array([[1.0, 0.0], [0.0, -1.0]]))


def bonds(N, periodic):
    """(i, j) nearest-neighbour pairs of the chain, in increasing i."""
    out = [(i, i + 1) for i in range(N - 1)]
    if periodic and N > 2:
        out.append((N - 1, 0))
    return out


def diagonal(spins, N, periodic, J=1.0):
    s = np.asarray(spins, dtype=np.float64)
    tot = np.zeros(s.shape[0])
    for i, j in bonds(N, periodic):
        tot += s[:, i] * s[:, j]
    return -J * tot


def flip(spin_row, i):
    s = np.array(spin_row, copy=True)
    s[i] = -s[i]
    return s


def eloc_naive(logpsi, spins, N, periodic, J=1.0, gamma=1.0,
               return_ratios=False):
    """Local energies of spins [B, N] for a batched log-psi callable: psi
    re-evaluated on every single-flip neighbour, the sum over the flipped
    site in increasing order, FP64."""
    spins = np.atleast_2d(spins)
    diag = diagonal(spins, N, periodic, J)
    seqs = []
    for b in range(spins.shape[0]):
        seqs.append(spins[b])
        for i in range(N):
            seqs.append(flip(spins[b], i))
    lps = logpsi(np.stack(seqs)).reshape(spins.shape[0], N + 1)
    E = np.empty(spins.shape[0])
    ratios = []
    for b in range(spins.shape[0]):
        r = np.exp(lps[b, 1:] - lps[b, 0])
        acc = 0.0
        for v in r:                          # flipped site order
            acc += v
        E[b] = diag[b] - gamma * acc
        ratios.append(r)
    return (E, ratios) if return_ratios else E


def eloc_network_naive(cfg, theta, spins, return_ratios=False):
    P = net.unpack(cfg, theta)
    return eloc_naive(net.logpsi_fn(cfg, P), spins, cfg.N, cfg.periodic,
                      cfg.J, cfg.gamma, return_ratios)


def _site_op(op, i, N):
    left = sp.identity(2 ** i, format="csr")
    right = sp.identity(2 ** (N - 1 - i), format="csr")
    return sp.kron(sp.kron(left, op, format="csr"), right, format="csr")


def hamiltonian(N, periodic, J=1.0, gamma=1.0):
    """Sparse H on 2^N states; site 0 is the most significant factor and
    spin +1 is |0> (Z = +1), as in oracle.ed."""
    H = sp.csr_matrix((2 ** N, 2 ** N))
    for i, j in bonds(N, periodic):
        H = H - J * (_site_op(_Z, i, N) @ _site_op(_Z, j, N))
    for i in range(N):
        H = H - gamma * _site_op(_X, i, N)
    return H.tocsr()


def ground_energy(N, periodic, J=1.0, gamma=1.0):
    vals = eigsh(hamiltonian(N, periodic, J, gamma), k=1, which="SA",
                 tol=1e-12)[0]
    return float(vals[0])


def all_states(N):
    return np.array(list(itertools.product([1, -1], repeat=N)),
                    dtype=np.int8)
