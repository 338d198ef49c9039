"""Oracle pins: lattice bookkeeping and the deduplicated evaluation (CPU).

* Bond set: 2N bonds periodic, 2L(L-1) open, every site of degree 4
  (periodic); neighbours are exactly the anti-aligned bonds and conserve Sz.
* The deduplicated local energy (Sec. 3.2) reproduces the naive
  re-evaluation of the same quantized network: every code identical, E_loc
  within 1e-10 relative, with and without certified code reuse; the changed
  row sets only grow with depth and start from the changed inputs.
"""
import numpy as np
import pytest

from oracle import eloc, lattice
from oracle import network as net
from workloads import (CONFIGS, make_params, make_spins, scale_codebooks,
                       with_batch)


@pytest.mark.parametrize("L", [3, 4, 5, 10, 16])
def test_bond_set(L):
    N = L * L
    bp = lattice.bonds(L, True)
    assert len(bp) == 2 * N
    deg = np.zeros(N, dtype=int)
    pairs = set()
    for b, i, j in bp:
        deg[i] += 1
        deg[j] += 1
        pairs.add((min(i, j), max(i, j)))
    assert (deg == 4).all() and len(pairs) == 2 * N
    assert [b for b, _, _ in bp] == sorted(b for b, _, _ in bp)
    assert len(lattice.bonds(L, False)) == 2 * L * (L - 1)
    with pytest.raises(ValueError):
        lattice.bonds(2, True)


def test_neighbours_and_diagonal():
    cfg = CONFIGS["large"]
    s = make_spins(cfg, batch=16)
    bl = lattice.bonds(cfg.L, True)
    diag = lattice.diagonal(s, bl)
    for b in range(16):
        nb = lattice.neighbours(s[b], bl)
        anti = sum(1 for _, i, j in bl if s[b, i] != s[b, j])
        assert len(nb) == anti
        assert diag[b] == 0.25 * (len(bl) - 2 * anti)
        for _, p1, p2 in nb:
            assert p1 < p2
            s2 = lattice.swap(s[b], p1, p2)
            assert s2.sum() == s[b].sum() and (s2 != s[b]).sum() == 2


def _check_dedup(cfg, batch, certified, alpha=1.0):
    cfg = with_batch(cfg, batch)
    theta = scale_codebooks(cfg, make_params(cfg), alpha)
    s = make_spins(cfg)
    En, ratios = eloc.eloc_network_naive(cfg, theta, s, return_ratios=True)
    Ed, info = eloc.eloc_dedup(cfg, theta, s, certified=certified,
                               return_info=True)
    assert np.allclose(Ed, En, rtol=1e-10, atol=0)
    r_naive = np.concatenate(ratios)
    r_dedup = np.array([r for _, r in info["ratios"]])
    assert np.allclose(r_dedup, r_naive, rtol=1e-10, atol=0)
    # codes identical to the naive full forward of every neighbour
    P = net.unpack(cfg, theta)
    bl = lattice.bonds(cfg.L, True)
    k = 0
    for b in range(batch):
        for _, p1, p2 in lattice.neighbours(s[b], bl):
            full = net.forward(cfg, P, lattice.swap(s[b], p1, p2)[None])
            assert np.array_equal(full["codes"][:, 0], info["codes"][k])
            sizes = info["changed"][k]
            assert sizes[0] in (1, 2)
            assert all(x <= y for x, y in zip(sizes, sizes[1:]))
            assert sizes[-1] <= cfg.N - (p1 + 1)
            k += 1
    return info


@pytest.mark.parametrize("certified", [False, True])
def test_dedup_equals_naive_small(certified):
    _check_dedup(CONFIGS["small"], 24, certified)


@pytest.mark.parametrize("certified", [False, True])
def test_dedup_equals_naive_medium(certified):
    _check_dedup(CONFIGS["medium"], 1, certified)


def test_certified_reuse_fires_on_insensitive_codes():
    """With codes far apart (codebooks scaled by 8) the certificate skips
    most searches, the changed sets stay near the two changed inputs, and
    the codes are still the naive ones."""
    cfg = with_batch(CONFIGS["medium"], 1, codebook_size=16)
    info = _check_dedup(cfg, 1, True, alpha=8.0)
    assert sum(info["vq_rows"]) < 0.5 * sum(info["att_rows"])
    assert np.mean([c[-1] for c in info["changed"]]) < 4


def test_dedup_with_attention_tail_equals_naive():
    """The deduplicated evaluation of a model ending with the attention-only
    half-block (every row from the first changed input recomputed there)
    equals the naive re-evaluation."""
    from dataclasses import replace
    cfg = replace(CONFIGS["small"], attn_tail=True, n_layers=2, batch=6)
    theta = make_params(cfg)
    s = make_spins(cfg)
    E_naive = eloc.eloc_network_naive(cfg, theta, s)
    E_dedup = eloc.eloc_dedup(cfg, theta, s)
    assert np.allclose(E_dedup, E_naive, rtol=1e-12, atol=0)
