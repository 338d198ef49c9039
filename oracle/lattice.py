"""Heisenberg model on an L x L square lattice (paper Sec. 4; k-local rows of
Sec. 2).

H = J * sum_<ij> S_i . S_j with S = sigma/2.  In the basis of z-spins
s_i in {+1,-1} one row of H has
  * a diagonal element (J/4) * sum_<ij> s_i s_j, and
  * one off-diagonal element per anti-aligned bond <ij> (k = 2, d = 2): the
    configuration with s_i and s_j exchanged.  Its value is +J/2, which the
    Marshall sign rotation (sign (-1)^{number of up spins on sublattice B},
    B = sites with r+c odd) turns into -J/2 on a bipartite lattice.

Bond order (canonical): bond b = 2*i + dir for site i = r*L + c, dir 0 links
(r, c) to (r, c+1 mod L), dir 1 links (r, c) to (r+1 mod L, c).  With open
boundaries the wrapping bonds are absent; the rest keep their ids.
"""
import numpy as np


def bonds(L, periodic=True):
    """List of (b, i, j) in increasing bond id b."""
    if periodic and L < 3:
        raise ValueError("periodic lattice needs L >= 3 (else bonds repeat)")
    out = []
    for r in range(L):
        for c in range(L):
            i = r * L + c
            if periodic or c + 1 < L:
                out.append((2 * i, i, r * L + (c + 1) % L))
            if periodic or r + 1 < L:
                out.append((2 * i + 1, i, ((r + 1) % L) * L + c))
    return out


def diagonal(spins, bond_list, J=1.0):
    """(J/4) sum_b s_i s_j for each row of spins [B, N]."""
    s = np.asarray(spins, dtype=np.float64)
    tot = np.zeros(s.shape[0])
    for _, i, j in bond_list:
        tot += s[:, i] * s[:, j]
    return 0.25 * J * tot


def neighbours(spin_row, bond_list):
    """Anti-aligned bonds of one configuration, in canonical order.

    Returns a list of (b, p1, p2) with p1 < p2 the two exchanged sites.
    """
    out = []
    for b, i, j in bond_list:
        if spin_row[i] != spin_row[j]:
            out.append((b, min(i, j), max(i, j)))
    return out


def swap(spin_row, i, j):
    s = np.array(spin_row, copy=True)
    s[i], s[j] = s[j], s[i]
    return s


def offdiag_element(J=1.0, marshall=True):
    return -0.5 * J if marshall else 0.5 * J
