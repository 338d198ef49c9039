"""GPU parity of the BF16 matrix-core path against the FP64 oracle.

The BF16 mode evaluates the network at bfloat16 parameters (the workloads
generate bfloat16-representable values, so the oracle sees the same ones),
with FP32 activations entering the matrix core as hi+lo bfloat16 pairs.

Every entry is compared with a hard bound; an entry beyond it must be a
proven quantizer near-tie (tests/near_tie.py): a code is an integer decided
by comparing floating-point distances, and where the two best codes are
closer than the path's rounding can resolve, the GPU's code is checked to
be nearest to its own attention output, whose distance from the oracle's
is no larger than that of the rows whose codes agree.

* log psi within 1e-3 of the oracle on every sequence whose codes all
  agree (observed errors are 1e-5: FP32 activations carry 2^-17 relative
  error from the hi/lo split, amplified through the layers).
* Neighbour ratios within RATIO_TOL = 1e-3 each (observed median 1e-5).
* Local energies within 1e-3 each and their mean within 1e-3, with the
  explained neighbours' terms taken out of both sides.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq
from oracle import eloc as oeloc
from oracle import lattice
from oracle import network as net
from workloads import CONFIGS, make_params, make_spins, with_batch

from gpu_common import dev_params, dev_spins, host, needs_gpu, say
from gpu_parity import adjusted_eloc, check_ratios, check_sequences

pytestmark = [pytest.mark.gpu, needs_gpu]

RATIO_TOL = 1e-3
LOGPSI_TOL = 1e-3
ELOC_TOL = 1e-3


@pytest.mark.parametrize("name,batch", [("medium", 64), ("large", 8),
                                        ("grad", 2)])
def test_forward_bf16(name, batch):
    mc = with_batch(CONFIGS[name], batch, precision="bf16")
    say(f"forward bf16 {name} B={batch}")
    theta = make_params(mc)
    s = make_spins(mc)
    P = net.unpack(mc, theta)
    cfg = vq.make_config(mc)
    p = dev_params(theta, "bf16")
    flips, ref = check_sequences(mc, P, cfg, p, s, LOGPSI_TOL)
    # vqnqs_forward_logpsi gives the same values as the activations call
    lp = host(vq.forward_logpsi(cfg, p, dev_spins(s)))
    lp2 = host(vq.forward_activations(cfg, p, dev_spins(s))[0])
    assert np.array_equal(lp, lp2)
    say(f"{len(flips)} of {batch} sequences with a proven near-tie")


def _eloc_every_neighbour(mc, theta, s, cfg, p, out):
    E, R = host(out["eloc"]), host(out["ratios"])
    P = net.unpack(mc, theta)
    bl = lattice.bonds(mc.L, mc.periodic)
    picks = [(b, range(len(lattice.neighbours(s[b], bl))))
             for b in range(s.shape[0])]
    rel, explained = check_ratios(mc, P, cfg, p, s, R, picks, RATIO_TOL)
    E_ref, r_ref = oeloc.eloc_network_naive(mc, theta, s, return_ratios=True)
    E_adj, E_ref_adj = adjusted_eloc(mc, E, E_ref, R, r_ref, explained)
    per = np.abs(E_adj - E_ref_adj) / np.abs(E_ref_adj)
    mean_adj = abs(E_adj.mean() - E_ref_adj.mean()) / abs(E_ref_adj.mean())
    mean_raw = abs(E.mean() - E_ref.mean()) / abs(E_ref.mean())
    say(f"{mc.name}: ratios median {np.median(rel):.2e}, {len(explained)} "
        f"explained; E_loc max {per.max():.2e}; mean energy raw "
        f"{mean_raw:.2e} adjusted {mean_adj:.2e}")
    assert per.max() < ELOC_TOL
    assert mean_adj < ELOC_TOL
    return explained


@pytest.mark.parametrize("flags", [0, vq.FLAG_CERTIFIED_VQ])
def test_local_energy_bf16_medium(flags):
    mc = with_batch(CONFIGS["medium"], 24, precision="bf16")
    say(f"eloc bf16 medium flags={flags}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc, flags=flags)
    p = dev_params(theta, "bf16")
    out = vq.local_energy(cfg, p, dev_spins(s), vq.DEDUP, ratios=True)
    _eloc_every_neighbour(mc, theta, s, cfg, p, out)


def test_local_energy_bf16_large_full_batch_sampled():
    """The benchmark's launch configuration (8192 samples, one call) with
    outputs of seeded samples and neighbours recomputed by the oracle (the
    first samples are compared in full against stored oracle values in
    test_gpu_large_golden.py)."""
    mc = CONFIGS["large"]
    say("eloc bf16 large full batch")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p = dev_params(theta, "bf16")
    ws = torch.empty(min(vq.workspace_size(cfg, mc.batch, vq.DEDUP, 0),
                         48 << 30), dtype=torch.uint8, device="cuda")
    out = vq.local_energy(cfg, p, dev_spins(s), vq.DEDUP, ratios=True,
                          counters=True, ws=ws)
    E, R = host(out["eloc"]), host(out["ratios"])
    ctr = host(out["counters"])
    del ws, out
    torch.cuda.empty_cache()
    assert ctr[vq.CTR["samples"]] == mc.batch
    P = net.unpack(mc, theta)
    bl = lattice.bonds(mc.L, True)
    rng = np.random.default_rng(11)
    picks = []
    for b in rng.choice(np.arange(16, mc.batch), 4, replace=False):
        nb = lattice.neighbours(s[b], bl)
        assert np.count_nonzero(R[b]) == len(nb)
        # E_loc assembly from the ratios: exact diagonal + (-J/2) sum
        diag = lattice.diagonal(s[b:b + 1], bl)[0]
        assert abs(E[b] - (diag - 0.5 * R[b].sum())) <= 1e-12 * abs(E[b])
        picks.append((int(b), sorted(rng.choice(len(nb), 3, replace=False))))
    rel, explained = check_ratios(mc, P, cfg, p, s, R, picks, RATIO_TOL)
    say(f"large sampled ratios: max {rel.max():.2e}, {len(explained)} "
        f"explained")


def test_plain_equals_dedup_large_bitwise_rows():
    mc = with_batch(CONFIGS["large"], 6, precision="bf16")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    ra = host(vq.local_energy(cfg, p, sp, vq.PLAIN, ratios=True)["ratios"])
    rb = host(vq.local_energy(cfg, p, sp, vq.DEDUP, ratios=True)["ratios"])
    rc = host(vq.local_energy(vq.make_config(mc, flags=1), p, sp, vq.DEDUP,
                              ratios=True)["ratios"])
    assert np.allclose(rb, ra, rtol=1e-12, atol=0)
    assert np.array_equal(rb, rc)


def test_max_lattice_32x32_bf16():
    """The largest lattice the library admits (32x32, 1024 sites): the
    matrix-core attention tiles would not fit in LDS, so the vector-unit
    attention serves.  Forward against the oracle, dedup equal to plain, and
    sampled ratios recomputed by the oracle."""
    mc = replace(CONFIGS["small"], name="max32", L=32, d_model=32, n_layers=1,
                 n_heads=2, d_ff=128, codebook_size=32, precision="bf16",
                 batch=2, spin_seed=1777)
    say("bf16 32x32")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    P = net.unpack(mc, theta)
    check_sequences(mc, P, cfg, p, s, LOGPSI_TOL)
    ra = host(vq.local_energy(cfg, p, sp, vq.PLAIN, ratios=True)["ratios"])
    rb = host(vq.local_energy(cfg, p, sp, vq.DEDUP, ratios=True)["ratios"])
    assert np.allclose(rb, ra, rtol=1e-12, atol=0)
    bl = lattice.bonds(mc.L, True)
    nb = lattice.neighbours(s[0], bl)
    assert np.count_nonzero(rb[0]) == len(nb)
    ks = [0, len(nb) // 3, 2 * len(nb) // 3, len(nb) - 1]
    check_ratios(mc, P, cfg, p, s, rb, [(0, ks)], RATIO_TOL)


@pytest.mark.parametrize("periodic,vq_heads", [(True, 4), (False, 1)],
                         ids=["periodic_H4", "open_H1"])
def test_bf16_quantizer_heads_and_open_boundary(periodic, vq_heads):
    """Matrix-core path with several quantizer heads (segment width 32) and
    with open boundaries: forward and local energies against the oracle,
    dedup equal to plain."""
    mc = replace(CONFIGS["small"], name="h4", L=6, d_model=128, n_layers=2,
                 n_heads=8, d_ff=512, codebook_size=64, vq_heads=vq_heads,
                 periodic=periodic, precision="bf16", batch=12,
                 spin_seed=1781)
    say(f"bf16 L6 periodic={periodic} H={vq_heads}")
    theta = make_params(mc)
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    P = net.unpack(mc, theta)
    check_sequences(mc, P, cfg, p, s, LOGPSI_TOL)
    a = vq.local_energy(cfg, p, sp, vq.PLAIN, ratios=True)
    b = vq.local_energy(cfg, p, sp, vq.DEDUP, ratios=True)
    assert np.allclose(host(b["ratios"]), host(a["ratios"]), rtol=1e-12, atol=0)
    _eloc_every_neighbour(mc, theta, s, cfg, p, b)


@pytest.mark.parametrize("vq_heads", [1, 4], ids=["H1", "H4"])
def test_bf16_duplicate_codewords_lowest_index(vq_heads):
    """Codebooks with exact duplicates, within a 16-code block (odd codes
    repeat the even ones) and across blocks (codes 16-31 repeat codes
    0-15): equal distances go to the lowest index (reading C2).  The
    neighbours' searches start from the sample's code and skip blocks that
    cannot hold the nearest one, the full sequences' searches do not; both
    must choose the same codes, so dedup equals plain, and the forward
    codes equal the oracle's on every sequence without a near-tie of
    distinct codewords."""
    from workloads.layout import param_layout
    mc = replace(CONFIGS["small"], name="dup", L=6, d_model=128, n_layers=2,
                 n_heads=8, d_ff=512, codebook_size=64, vq_heads=vq_heads,
                 precision="bf16", batch=8, spin_seed=1791)
    say(f"bf16 duplicate codewords H={vq_heads}")
    theta = make_params(mc)
    for name, shape, kind, off, n in param_layout(mc):
        if name.endswith(".codebook"):
            cb = theta[off:off + n].reshape(shape)
            cb[:, 1::2] = cb[:, 0::2]
            cb[:, 16:32] = cb[:, 0:16]
            theta[off:off + n] = cb.ravel()
    s = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(s)
    P = net.unpack(mc, theta)
    flips, ref = check_sequences(mc, P, cfg, p, s, LOGPSI_TOL)
    _, cd, _ = vq.forward_activations(cfg, p, sp)
    cd = host(cd)
    # every chosen code is the lowest index of its duplicate class
    assert (cd % 2 == 0).all() and not ((cd >= 16) & (cd < 32)).any()
    a = vq.local_energy(cfg, p, sp, vq.PLAIN, ratios=True)
    b = vq.local_energy(cfg, p, sp, vq.DEDUP, ratios=True)
    assert np.array_equal(host(b["ratios"]), host(a["ratios"]))
    assert np.array_equal(host(b["eloc"]), host(a["eloc"]))
    _eloc_every_neighbour(mc, theta, s, cfg, p, b)
