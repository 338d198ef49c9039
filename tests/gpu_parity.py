"""Parity checks shared by the GPU tests: results of the library against
the FP64 oracle, entry by entry, where every entry beyond its tolerance
must be a proven quantizer near-tie (tests/near_tie.py)."""
import numpy as np

import paper_2212_11296_amd as vq
from oracle import lattice
from oracle import network as net
from oracle import tfim
from workloads import param_layout

from gpu_common import dev_spins, host, say
from near_tie import explain


def codebooks(P):
    return [lay["codebook"] for lay in P["layers"]]


def check_sequences(mc, P, cfg, p, seqs, logpsi_tol):
    """GPU forward (codes, attention outputs, log psi) of seqs against the
    oracle: every sequence whose codes all agree has log psi within
    logpsi_tol; every other one is a proven near-tie at the first layer
    where the codes part.  Returns the indices of the near-tie sequences and
    the oracle forward."""
    lp, cd, at = vq.forward_activations(cfg, p, dev_spins(seqs))
    lp, cd, at = host(lp), host(cd), host(at)
    ref = net.forward(mc, P, seqs, keep=True)
    ocd = np.transpose(ref["codes"], (1, 0, 2, 3))
    cbs = codebooks(P)
    flips = []
    for b in range(seqs.shape[0]):
        oa = np.stack([c["a"][b] for c in ref["caches"]])
        ex = explain(cbs, cd[b], at[b], ocd[b], oa)
        if ex is None:
            assert abs(lp[b] - ref["logpsi"][b]) < logpsi_tol, \
                (b, lp[b], ref["logpsi"][b])
        else:
            assert ex["ok"], (b, ex)
            flips.append(b)
    return flips, ref


def check_ratios(mc, P, cfg, p, spins, R, picks, tol):
    """Compares R[b][k] with the oracle for (b, ks) in picks; an entry beyond
    tol must come from a proven near-tie of the neighbour's or the sample's
    codes.  Returns (relative errors, explained (b, k) pairs).  Neighbour k
    is the k-th swapped antiparallel bond of the Heisenberg lattice, or the
    flip of site k on the transverse-field Ising chain."""
    chain = mc.hamiltonian == "tfim"
    bl = None if chain else lattice.bonds(mc.L, mc.periodic)
    seqs, owner = [], []
    for b, ks in picks:
        nb = None if chain else lattice.neighbours(spins[b], bl)
        seqs.append(spins[b])
        owner.append((b, -1))
        for k in ks:
            seqs.append(tfim.flip(spins[b], k) if chain else
                        lattice.swap(spins[b], nb[k][1], nb[k][2]))
            owner.append((b, k))
    seqs = np.stack(seqs)
    ref = net.forward(mc, P, seqs, keep=True)
    lp0 = {b: ref["logpsi"][j] for j, (b, k) in enumerate(owner) if k < 0}
    rel = np.array([abs(R[b, k] / np.exp(ref["logpsi"][j] - lp0[b]) - 1)
                    if k >= 0 else 0.0 for j, (b, k) in enumerate(owner)])
    bad = [j for j, (b, k) in enumerate(owner) if k >= 0 and rel[j] > tol]
    explained = []
    if bad:
        idx = sorted(set(bad) | {owner.index((owner[j][0], -1)) for j in bad})
        _, gcd, gat = vq.forward_activations(cfg, p, dev_spins(seqs[idx]))
        gcd, gat = host(gcd), host(gat)
        ocd = np.transpose(ref["codes"], (1, 0, 2, 3))
        cbs = codebooks(P)
        pos = {j: i for i, j in enumerate(idx)}
        for j in bad:
            b, k = owner[j]
            js = owner.index((b, -1))
            exs = []
            for jj in (js, j):
                oa = np.stack([c["a"][jj] for c in ref["caches"]])
                exs.append(explain(cbs, gcd[pos[jj]], gat[pos[jj]], ocd[jj],
                                   oa))
            say(f"{mc.name} ({b},{k}) rel err {rel[j]:.3e}: {exs}")
            found = [e for e in exs if e is not None]
            assert found, f"unexplained ratio error at {(b, k)}: {rel[j]}"
            assert all(e["ok"] for e in found), ((b, k), found)
            explained.append((b, k))
    return rel[[k >= 0 for _, k in owner]], explained


def adjusted_eloc(mc, E, E_ref, R, r_ref, explained):
    """Local energies of both sides with the explained neighbours' terms
    taken out (a near-tie resolved the other way is a different valid
    answer).  r_ref[b][k] are the oracle's ratios."""
    h = -0.5 * mc.J
    E_adj, E_ref_adj = np.array(E, dtype=float), np.array(E_ref, dtype=float)
    for b, k in explained:
        E_adj[b] -= h * R[b, k]
        E_ref_adj[b] -= h * r_ref[b][k]
    return E_adj, E_ref_adj


# Gradient tolerances per parameter tensor: its largest entry error over its
# largest reference entry (FP32; BF16, whose forward and recompute run on
# the matrix core at the hi/lo split's 2^-17).
FP32_BLOCK_TOL = 1e-4
BF16_BLOCK_TOL = 1e-2


def check_blocks(mc, g, ref, tol, label=""):
    """Every parameter tensor separately: largest entry error over the
    tensor's largest reference entry below tol (a tensor whose reference is
    exactly zero must come out exactly zero)."""
    worst = ("", 0.0)
    for name, shape, kind, off, n in param_layout(mc):
        a, b = g[off:off + n], ref[off:off + n]
        scale = np.abs(b).max()
        if scale == 0.0:
            assert not np.any(a), (label, name)
            continue
        e = np.abs(a - b).max() / scale
        if e > worst[1]:
            worst = (name, e)
        assert e < tol, (label, name, e)
    say(f"{label} worst tensor {worst[0]}: {worst[1]:.2e}")
