"""BF16 parity at the 16x16 workload (d=128, 8 layers, 8 heads, MLP 512,
Q=1024) in the benchmark's launch configuration: the whole batch of 8192
samples in one vqnqs_local_energy call (dedup), with the same workspace
cap as the benchmark, compared entry by entry with FP64 oracle values of
the first samples (tests/golden/large_bf16_eloc.json, written by
tests/golden/make_large_goldens.py from oracle/ alone).

* Every neighbour ratio psi(s')/psi(s) of every golden sample: relative
  error at most RATIO_TOL = 1e-3, unless the GPU's codes for s' (or s)
  differ from the oracle's and every differing code at the first layer
  where they part is a proven near-tie (tests/near_tie.py: the GPU's code
  is nearest to its own attention output within the kernel's score error,
  and its attention output is no further from the oracle's than that of
  the rows whose codes agree).  An entry beyond RATIO_TOL that is not so
  explained fails.  RATIO_TOL is the precision target of this path.
* The codes of every golden sample s against the oracle's, with the same
  rule for differences.
* Local energy of eq. (2): per sample within 1e-3 relative once the
  contributions of the explained neighbours are taken out of both sides
  (a near-tie resolved the other way is a different, equally valid
  answer), and the mean over the samples within 1e-3 relative, both with
  and without that adjustment reported; the adjusted mean is asserted.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq
from oracle import lattice
from oracle import network as net
from workloads import CONFIGS, make_params, make_spins

from gpu_common import dev_params, dev_spins, host, needs_gpu, say
from near_tie import explain

pytestmark = [pytest.mark.gpu, needs_gpu]

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "large_bf16_eloc.json")
RATIO_TOL = 1e-3
ELOC_TOL = 1e-3
WS_CAP = 192 << 30           # the benchmark's workspace cap (8 chunks)


def _codebooks(mc, P):
    return [lay["codebook"] for lay in P["layers"]]


def test_large_bf16_every_neighbour_against_oracle_goldens():
    with open(GOLD) as f:
        gold = json.load(f)
    mc = CONFIGS["large"]
    # the workload the values were written for (fields added later keep
    # their defaults)
    assert all(mc.as_dict()[k] == v for k, v in gold["workload"].items())
    assert mc.hamiltonian == "heisenberg"
    G = gold["samples"]
    nS = len(G)
    say(f"large bf16 golden: full batch {mc.batch}, {nS} golden samples")
    theta = make_params(mc)
    spins = make_spins(mc)
    cfg = vq.make_config(mc)
    p, sp = dev_params(theta, "bf16"), dev_spins(spins)
    need = vq.workspace_size(cfg, mc.batch, vq.DEDUP, 0)
    ws = torch.empty(min(need, WS_CAP), dtype=torch.uint8, device="cuda")
    out = vq.local_energy(cfg, p, sp, vq.DEDUP, ratios=True, ws=ws)
    E = host(out["eloc"])[:nS]
    R = host(out["ratios"])[:nS]
    del ws, out
    torch.cuda.empty_cache()
    P = net.unpack(mc, theta)
    cbs = _codebooks(mc, P)
    bl = lattice.bonds(mc.L, mc.periodic)

    # codes of the samples themselves
    lp_s, codes_s, attn_s = vq.forward_activations(cfg, p, sp[:nS])
    codes_s, attn_s = host(codes_s), host(attn_s)
    sample_flip = {}
    for b, g in enumerate(G):
        oc = np.asarray(g["codes"])                      # [nl][N][H]
        if not np.array_equal(codes_s[b], oc):
            ref = net.forward(mc, P, spins[b:b + 1], keep=True)
            oa = np.stack([c["a"][0] for c in ref["caches"]])
            ex = explain(cbs, codes_s[b], attn_s[b], oc, oa)
            say(f"sample {b}: code difference {ex}")
            assert ex["ok"], (b, ex)
            sample_flip[b] = ex

    # every ratio
    rel_all, outliers = [], []
    for b, g in enumerate(G):
        nb = lattice.neighbours(spins[b], bl)
        assert [x[0] for x in nb] == g["bonds"]
        r_o = np.asarray(g["ratios"])
        assert np.count_nonzero(R[b]) == len(r_o)
        rel = np.abs(R[b, :len(r_o)] / r_o - 1.0)
        rel_all.append(rel)
        for k in np.nonzero(rel > RATIO_TOL)[0]:
            outliers.append((b, int(k)))
    rel_all = np.concatenate(rel_all)
    say(f"ratios: n={rel_all.size} median={np.median(rel_all):.2e} "
        f"p99={np.quantile(rel_all, 0.99):.2e} max={rel_all.max():.2e} "
        f"above {RATIO_TOL}: {len(outliers)}")

    # every entry beyond the tolerance must come from a proven near-tie of
    # the neighbour (or of its sample)
    # (a sample whose own codes part from the oracle's has every ratio
    # shifted by its log psi: all of its neighbours count as explained)
    explained = {(b, k) for b in sample_flip
                 for k in range(len(G[b]["ratios"]))}
    todo = [(b, k) for b, k in outliers if b not in sample_flip]
    if todo:
        seqs = np.stack([lattice.swap(spins[b], *lattice.neighbours(
            spins[b], bl)[k][1:]) for b, k in todo])
        _, gcd, gat = vq.forward_activations(cfg, p, dev_spins(seqs))
        gcd, gat = host(gcd), host(gat)
        ref = net.forward(mc, P, seqs, keep=True)
        ocd = np.transpose(ref["codes"], (1, 0, 2, 3))     # [S][nl][N][H]
        for j, (b, k) in enumerate(todo):
            oa = np.stack([c["a"][j] for c in ref["caches"]])
            ex = explain(cbs, gcd[j], gat[j], ocd[j], oa)
            say(f"neighbour ({b},{k}) rel err "
                f"{abs(R[b, k] / G[b]['ratios'][k] - 1):.3e}: {ex}")
            assert ex is not None, f"unexplained ratio error at {(b, k)}"
            assert ex["ok"], ((b, k), ex)
            explained.add((b, k))

    # local energies: the explained neighbours' terms out of both sides
    h = -0.5 * mc.J
    E_o = np.array([g["eloc"] for g in G])
    E_g_adj, E_o_adj = E.copy(), E_o.copy()
    for b, k in explained:
        E_g_adj[b] -= h * R[b, k]
        E_o_adj[b] -= h * G[b]["ratios"][k]
    per = np.abs(E_g_adj - E_o_adj) / np.abs(E_o_adj)
    mean_raw = abs(E.mean() - E_o.mean()) / abs(E_o.mean())
    mean_adj = abs(E_g_adj.mean() - E_o_adj.mean()) / abs(E_o_adj.mean())
    say(f"E_loc: per-sample rel err (adjusted) median={np.median(per):.2e} "
        f"max={per.max():.2e}; mean energy rel err raw={mean_raw:.2e} "
        f"adjusted={mean_adj:.2e}; {len(explained)} explained neighbours")
    assert per.max() < ELOC_TOL
    assert mean_adj < ELOC_TOL
