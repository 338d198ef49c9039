#!/usr/bin/env python3
"""Writes tests/golden/large_bf16_eloc.json: FP64 oracle values for the
first samples of the 16x16 BF16 workload (periodic Heisenberg, d=128,
8 layers, 8 heads, MLP 512, Q=1024; parameters rounded to bfloat16 as the
workload generator makes them).

Per sample: log psi, the quantizer codes of every layer and position, the
exact diagonal, and for every exchange neighbour in bond order its bond,
log psi and psi(s')/psi(s) = exp(log psi(s') - log psi(s)); the local
energy of eq. (2) and the mean over the samples.  Everything comes from
oracle/ (plain re-evaluation of every neighbour, eq. 2) and workloads/.

    python tests/golden/make_large_goldens.py [--samples 16]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(
    os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lattice                       # noqa: E402
from oracle import network as net                # noqa: E402
from workloads import CONFIGS, make_params, make_spins   # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                   "large_bf16_eloc.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=16)
    args = ap.parse_args()
    mc = CONFIGS["large"]
    theta = make_params(mc)
    spins = make_spins(mc)[:args.samples]
    P = net.unpack(mc, theta)
    bl = lattice.bonds(mc.L, mc.periodic)
    diag = lattice.diagonal(spins, bl, mc.J)
    h_off = lattice.offdiag_element(mc.J, mc.marshall)
    lp_fn = net.logpsi_fn(mc, P, chunk=32)
    samples = []
    t0 = time.time()
    for b in range(spins.shape[0]):
        base = net.forward(mc, P, spins[b:b + 1])
        lp0 = float(base["logpsi"][0])
        nb = lattice.neighbours(spins[b], bl)
        seqs = np.stack([lattice.swap(spins[b], p1, p2) for _, p1, p2 in nb])
        lps = lp_fn(seqs)
        r = np.exp(lps - lp0)
        acc = 0.0
        for v in r:                                  # bond order
            acc += v
        samples.append({
            "index": b,
            "logpsi": lp0,
            "codes": base["codes"][:, 0, :, :].astype(int).tolist(),
            "diag": float(diag[b]),
            "bonds": [int(x[0]) for x in nb],
            "logpsi_nb": [float(x) for x in lps],
            "ratios": [float(x) for x in r],
            "eloc": float(diag[b] + h_off * acc),
        })
        print(f"sample {b}: {len(nb)} neighbours, E_loc "
              f"{samples[-1]['eloc']:.6f} ({time.time() - t0:.0f} s)",
              flush=True)
    doc = {
        "what": "FP64 oracle (plain re-evaluation, eq. 2) on the first "
                f"{len(samples)} samples of the 16x16 BF16 workload",
        "workload": mc.as_dict(),
        "generator": "tests/golden/make_large_goldens.py",
        "mean_eloc": float(np.mean([s["eloc"] for s in samples])),
        "samples": samples,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
