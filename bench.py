#!/usr/bin/env python3
"""Local-energy throughput of the VQ-NQS path on one MI355X.

One step = one vqnqs_local_energy call (deduplicated form) over the whole
batch of the large workload: 16x16 periodic Heisenberg lattice, transformer
d=128, 8 layers, 8 heads, MLP 512, codebook 1024, 8192 seeded Sz=0 samples,
BF16 matrix-core products with FP32 accumulation and FP64 ratios/sums.
Inputs (parameters, spins, workspace) are resident in HBM before timing.

Also measured in the same run: the plain full-recompute form on the same
inputs (the comparator), per-kernel device time from the library's HIP-event
timing on its launch stream (roofline of the dominant kernel), and the CPU
oracle on a bounded sample (cpu_baseline).  Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

METRIC = ("local-energy evals/sec, VQ-dedup vs plain on 1 MI355X, at "
          "≤1e-3 rel err")
UNIT = "local-energy evals/s"
PEAK = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}     # TFLOP/s, dense
HBM_PEAK = 8000.0                                         # GB/s
# Attention at head width 16-32 has a second, tighter bound than the matrix
# core: every (query, key) pair needs one exponential on the vector unit.
# The bench measures the device's exponential issue rate live
# (vqnqs_probe_exp_rate: independent v_exp_f32 chains on every SIMD) and
# reports the attention kernel against it beside the matrix-core roofline;
# the exponential bound in FLOP/s is that rate times the algorithmic FLOPs
# of a pair (4 d_head: q.k and p.v).
TRAFFIC_FILE = "profiles/attention_dedup_16x16_bf16__hbm_traffic.json"
GOLDEN_FILE = "tests/golden/large_bf16_eloc.json"


def flops_model(mc, ctr, base_samples):
    """Algorithmic FLOPs per kernel class (2 FLOP per multiply-add) from the
    library's work counters.  The hi/lo second matrix-core pass is not
    counted: it is an implementation cost, not algorithmic work."""
    d, F, Q, N, nh = (mc.d_model, mc.d_ff, mc.codebook_size, mc.N,
                      mc.n_heads)
    dh = d // nh
    pairs_total = ctr["attn_pairs"]
    pairs_base = base_samples * mc.n_layers * nh * N * (N + 1) // 2
    return {
        "qkv": 2.0 * ctr["qkv_rows"] * d * 3 * d,
        "mlp": 2.0 * ctr["mlp_rows"] * 2 * d * F,
        "vq": 2.0 * ctr["vq_rows"] * Q * d,
        "attention_seq": 4.0 * pairs_base * dh,
        "attention_dedup": 4.0 * max(pairs_total - pairs_base, 0) * dh,
        "head": 2.0 * ctr["head_rows"] * d * 2,
    }


def kernel_source_digest():
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       "paper_2212_11296_amd", "csrc", "kernels_attn.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel, mc, launches_per_call):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated),
    or None when the summary is absent, covers another kernel or workload,
    was taken with another split of the batch into launches (the bytes of
    one launch depend on it), or from a different kernel source."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        TRAFFIC_FILE)
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel") != kernel or t.get("L") != mc.L
            or t.get("batch") != mc.batch
            or t.get("launches_per_call") != launches_per_call
            or t.get("source_sha256") != kernel_source_digest()):
        return None
    return t.get("bytes_per_launch")


def golden_parity(mc, out):
    """Errors of this run's results against the committed FP64 oracle
    values of the first samples (tests/golden, written from oracle/ only):
    every neighbour ratio and local energy of those samples and their mean
    energy.  None when the file covers another workload."""
    import numpy as np
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        GOLDEN_FILE)
    try:
        with open(path) as f:
            gold = json.load(f)
    except (OSError, ValueError):
        return None
    w = gold.get("workload", {})
    if (w.get("L") != mc.L or w.get("d_model") != mc.d_model
            or w.get("n_layers") != mc.n_layers
            or w.get("codebook_size") != mc.codebook_size
            or w.get("spin_seed") != mc.spin_seed
            or w.get("param_seed") != mc.param_seed
            or w.get("precision") != mc.precision):
        return None
    G = gold["samples"]
    n = len(G)
    E = out["eloc"][:n].cpu().numpy()
    R = out["ratios"][:n].cpu().numpy()
    rel = np.concatenate([np.abs(R[b, :len(g["ratios"])]
                                 / np.asarray(g["ratios"]) - 1.0)
                          for b, g in enumerate(G)])
    E_o = np.array([g["eloc"] for g in G])
    per = np.abs(E - E_o) / np.abs(E_o)
    return {
        "samples": n, "ratios": int(rel.size),
        "ratio_rel_err": {"median": float(np.median(rel)),
                          "p99": float(np.quantile(rel, 0.99)),
                          "max": float(rel.max()),
                          "n_above_1e-3": int((rel > 1e-3).sum())},
        "eloc_rel_err": {"median": float(np.median(per)),
                         "max": float(per.max()),
                         "n_above_1e-3": int((per > 1e-3).sum())},
        "mean_energy_rel_err": float(abs(E.mean() - E_o.mean())
                                     / abs(E_o.mean())),
        "note": "raw comparison; entries beyond 1e-3 are checked as "
                "quantizer near-ties by tests/test_gpu_large_golden.py",
    }


def counters_dict(vq, arr, nl):
    out = {k: int(arr[v]) for k, v in vq.CTR.items() if k != "changed0"}
    out["changed"] = [int(arr[vq.CTR["changed0"] + l]) for l in range(nl + 1)]
    return out


def cpu_baseline(mc, theta, spins, gpu_ratios, n_nb0, budget_s):
    """Times the FP64 oracle (plain re-evaluation, eq. 2) on a bounded sample:
    log psi of sample 0 and of its first k neighbours; the rate is scaled to
    whole local energies with sample 0's neighbour count.  The same ratios
    are compared with the GPU's as an accuracy spot check."""
    import numpy as np
    from oracle import lattice
    from oracle import network as onet
    from oracle import tfim
    P = onet.unpack(mc, theta)
    if mc.hamiltonian == "tfim":
        nbs = [tfim.flip(spins[0], i) for i in range(mc.N)]
    else:
        bl = lattice.bonds(mc.L, mc.periodic)
        nbs = [lattice.swap(spins[0], p1, p2)
               for _, p1, p2 in lattice.neighbours(spins[0], bl)]
    t0 = time.perf_counter()
    lp0 = onet.forward(mc, P, spins[0:1])["logpsi"][0]
    per = time.perf_counter() - t0
    k = int(max(4, min(len(nbs), budget_s / max(per, 1e-3))))
    t0 = time.perf_counter()
    sub = np.stack(nbs[:k])
    lps = onet.logpsi_fn(mc, P, chunk=32)(sub)
    dt = time.perf_counter() - t0 + per
    r_ref = np.exp(lps - lp0)
    rel = np.abs(gpu_ratios[:k] / r_ref - 1.0)
    # a quantizer near-tie resolved to the other code moves a ratio by a
    # finite step: the maximum alone does not describe the accuracy
    err = {"n": int(k), "median": float(np.median(rel)),
           "p99": float(np.quantile(rel, 0.99)), "max": float(np.max(rel)),
           "n_above_1e-3": int((rel > 1e-3).sum())}
    evals_per_eloc = 1 + n_nb0
    rate = (k + 1) / dt / evals_per_eloc
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        th = [i.get("num_threads") for i in threadpool_info()
              if i.get("user_api") == "blas"]
        if th:
            cores = int(th[0])
    except Exception:
        pass
    out = {"value": rate, "unit": UNIT, "cores": cores, "kind": "oracle",
           "sample": (f"sample 0 of the batch: log psi of the sample and of "
                      f"its first {k} of {len(nbs)} neighbours, "
                      f"NumPy float64, {dt:.1f} s; rate scaled by "
                      f"1 + n_neighbours evaluations per local energy")}
    # the oracle's deduplicated form (Sec. 3.2) on the same sample, when the
    # plain one left time for it: one whole local energy
    if mc.hamiltonian != "tfim" and dt < budget_s:
        from oracle import eloc as oeloc
        t0 = time.perf_counter()
        E_d = oeloc.eloc_dedup(mc, theta, spins[0:1])[0]
        dt_d = time.perf_counter() - t0
        out["dedup"] = {"value": 1.0 / dt_d, "unit": UNIT, "kind": "oracle",
                        "sample": (f"sample 0: the oracle's deduplicated "
                                   f"local energy over all {len(nbs)} "
                                   f"neighbours, {dt_d:.1f} s"),
                        "eloc": float(E_d)}
    return out, err


def grad_flops(mc):
    """Algorithmic FLOPs of the gradient's products per sample (2 per
    multiply-add): the recomputed MLP input product and the backward
    products of every layer (MLP, output projection, quantizer, QKV)."""
    N, d, F, Q = mc.N, mc.d_model, mc.d_ff, mc.codebook_size
    per_layer = 10 * N * d * F + 16 * N * d * d + 6 * N * Q * d
    return {"grad_gemm": float(mc.n_layers * per_layer),
            "grad_attention": float(mc.n_layers * 8 * N * N * mc.d_head
                                    * mc.n_heads)}


def bench_grad(args, vq, torch, np, mc, make_params, make_spins):
    """Weighted straight-through gradient sum_i w_i d log psi_i / d theta of
    the 20x20 gradient workload; prints one JSON line."""
    B = mc.batch
    dev = torch.device("cuda:0")
    theta = make_params(mc)
    spins = make_spins(mc)
    p = torch.tensor(theta, dtype=torch.float32, device=dev)
    sp = torch.tensor(spins, device=dev)
    w = torch.tensor(np.random.default_rng(77).standard_normal(B),
                     dtype=torch.float64, device=dev)
    cfg = vq.make_config(mc)
    need = vq.workspace_size(cfg, B, vq.WS_GRAD, 0)
    ws = torch.empty(min(need, int(args.ws_gb * (1 << 30))),
                     dtype=torch.uint8, device=dev)
    g = torch.empty(p.numel(), dtype=torch.float32, device=dev)

    def step():
        vq.grad_logpsi(cfg, p, sp, weights=w, ws=ws, check=False, out=g)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    vq.profile_reset()
    vq.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    vq.profile_enable(False)
    ms = e0.elapsed_time(e1) / args.steps
    prof = vq.profile_read()
    vq.api._check_status(ws)
    per_kernel = {k: {"ms_per_step": v[0] / args.steps,
                      "launches_per_step": v[1] / args.steps}
                  for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    dom = next(iter(per_kernel))
    fl = {k: v * B for k, v in grad_flops(mc).items()}
    roof = {"bound": None, "kernel": dom, "achieved": None, "peak": None,
            "unit": None, "frac": None, "traffic": None}
    if dom in fl:
        launches = prof[dom][1]
        per_launch = fl[dom] * args.steps / launches
        avg = prof[dom][0] / launches
        ach = per_launch / (avg / 1e3) / 1e12
        if dom == "grad_attention":
            bound, peak = "alu", PEAK["fp32"]
        else:
            # FP32-accurate products (three bf16 matrix-core passes): the
            # FP32 dense matrix peak
            bound, peak = "mfma", PEAK["fp32"]
        roof = {"bound": bound, "kernel": dom, "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                "flop_per_launch": per_launch, "avg_launch_ms": avg}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import grad as og
        t0 = time.perf_counter()
        k = 0
        while k < 1 or (time.perf_counter() - t0 < args.cpu_seconds and k < 4):
            og.grad_logpsi(mc, theta, spins[k:k + 1])
            k += 1
        dt = time.perf_counter() - t0
        try:
            cores = len(os.sched_getaffinity(0))
        except AttributeError:
            cores = os.cpu_count()
        cpu = {"value": k / dt, "unit": "samples/s", "cores": cores,
               "kind": "oracle",
               "sample": f"per-sample gradients of the first {k} samples, "
                         f"torch float64 autograd on the CPU, {dt:.1f} s"}
    res = {
        "metric": "straight-through gradient samples/sec (weighted sum of "
                  "d log psi / d theta), 1 MI355X",
        "value": B / (ms / 1000.0), "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": (f"{mc.L}x{mc.L} periodic Heisenberg, VQ "
                                f"transformer d={mc.d_model} L={mc.n_layers} "
                                f"heads={mc.n_heads} mlp={mc.d_ff} "
                                f"Q={mc.codebook_size}, {B} seeded Sz=0 "
                                f"samples, weighted gradient"),
                   "L": mc.L, "batch": B, "precision": mc.precision},
        "roofline": roof, "cpu_baseline": cpu,
        "algorithmic_tflop_per_step": sum(fl.values()) / 1e12,
        "kernels": per_kernel,
    }
    print(json.dumps(res))


def bench_multi(args, vq, torch, np, make_params, make_spins, with_batch):
    """Mixed-lattice batch (6x6 .. 20x20, one model each, 512 .. 8192
    samples): one vqnqs_local_energy_multi call per step, replayed as a
    captured graph, against one vqnqs_local_energy call per lattice."""
    from workloads import MULTI_LATTICE
    dev = torch.device("cuda:0")
    jobs = []
    mix = MULTI_LATTICE
    if args.batch:
        # the same lattices and models with this many samples each: a mix in
        # which no single lattice fills the device
        mix = [with_batch(mc, args.batch) for mc in MULTI_LATTICE]
    for mc in mix:
        jobs.append((vq.make_config(mc),
                     torch.tensor(make_params(mc), dtype=torch.float32,
                                  device=dev),
                     torch.tensor(make_spins(mc), device=dev)))
    total = sum(int(s.shape[0]) for _, _, s in jobs)
    need = vq.workspace_size_multi(jobs)
    ws = torch.empty(min(need, int(args.ws_gb * (1 << 30))),
                     dtype=torch.uint8, device=dev)
    # launch choices for this model width, tuned on the 16x16 lattice
    cfg16, p16, s16 = jobs[3]
    tune_ws = torch.empty(vq.workspace_size(cfg16, 512, vq.DEDUP, 0)
                          + 8 * 512 + 256, dtype=torch.uint8, device=dev)
    if args.tuning_cache:
        from paper_2212_11296_amd import tuning
        choices, _ = tuning.autotune_cached(cfg16, p16, s16[:512],
                                            args.tuning_cache, ws=tune_ws)
    else:
        choices = vq.autotune(cfg16, p16, s16[:512], ws=tune_ws)
    del tune_ws
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    flags = vq.MULTI_CONCURRENT | vq.MULTI_GRAPH
    outs = vq.local_energy_multi(jobs, flags=flags, ws=ws, check=False)
    for _ in range(args.warmup):
        vq.local_energy_multi(jobs, flags=flags, ws=ws, outs=outs, check=False)
    torch.cuda.synchronize()
    times = []
    e_all0, e_all1 = ev(), ev()
    e_all0.record(stream)
    for _ in range(args.steps):
        a, b = ev(), ev()
        a.record(stream)
        vq.local_energy_multi(jobs, flags=flags, ws=ws, outs=outs, check=False)
        b.record(stream)
        times.append((a, b))
    e_all1.record(stream)
    torch.cuda.synchronize()
    vq.api._check_status(ws)
    ms = e_all0.elapsed_time(e_all1) / args.steps
    lat = sorted(a.elapsed_time(b) for a, b in times)
    pct = lambda q: lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]
    # the same lattices one call at a time on one stream
    e0, e1 = ev(), ev()
    e0.record(stream)
    per = []
    for cfg, p, s in jobs:
        a, b = ev(), ev()
        a.record(stream)
        vq.local_energy(cfg, p, s, vq.DEDUP, ws=ws, check=False)
        b.record(stream)
        per.append((a, b))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1)
    res = {
        "metric": "local-energy evals/sec, mixed-lattice batch (6x6..20x20) "
                  "in one graph-replayed multi-lattice call, 1 MI355X",
        "value": total / (ms / 1000.0), "unit": "local-energy evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "lattices 6x6/8x8/12x12/16x16/20x20 with "
                               + ("/".join(str(int(j[2].shape[0]))
                                           for j in jobs))
                               + " seeded Sz=0 samples, "
                               "one VQ transformer each (d=128, 6 layers, "
                               "8 heads, MLP 512, Q=512), dedup local energy",
                   "samples": total, "flags": flags},
        "latency_ms": {"p50": pct(0.5), "p99": pct(0.99), "all": lat},
        "sequential_single_calls": {
            "value": total / (ms_seq / 1000.0), "ms": ms_seq,
            "per_lattice_ms": {f"{cfg.L}x{cfg.L}": a.elapsed_time(b)
                               for (cfg, _, _), (a, b) in zip(jobs, per)}},
        "speedup_vs_sequential": ms_seq / ms,
        "tuning": {"qkv_mb": choices[0], "mlp_mb": choices[1],
                   "vq_mb": choices[2]},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(res))


def bench_sample(args, vq, torch, np, mc, make_params):
    """Direct autoregressive sampling (chain rule) of the whole batch of
    the workload, uniform numbers resident in HBM; one JSON line."""
    B, N = mc.batch, mc.N
    dev = torch.device("cuda:0")
    theta = make_params(mc)
    dt_param = torch.float64 if mc.precision == "f64" else torch.float32
    p = torch.tensor(theta, dtype=dt_param, device=dev)
    cfg = vq.make_config(mc)
    u = torch.rand((B, N), dtype=torch.float64,
                   generator=torch.Generator().manual_seed(5)).to(dev)
    need = vq.workspace_size(cfg, B, vq.WS_SAMPLE, 0)
    ws = torch.empty(min(need, int(args.ws_gb * (1 << 30))),
                     dtype=torch.uint8, device=dev)
    out = {"spins": torch.empty((B, N), dtype=torch.int8, device=dev),
           "logpsi": torch.empty(B, dtype=torch.float64, device=dev)}
    for _ in range(args.warmup):
        vq.sample(cfg, p, u, ws=ws, check=False, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    vq.profile_reset()
    vq.profile_enable(True)
    e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    e0.record(stream)
    for _ in range(args.steps):
        vq.sample(cfg, p, u, ws=ws, check=False, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    vq.profile_enable(False)
    ms = e0.elapsed_time(e1) / args.steps
    prof = vq.profile_read()
    vq.api._check_status(ws)
    per_kernel = {k: {"ms_per_step": v[0] / args.steps,
                      "launches_per_step": v[1] / args.steps}
                  for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    # the forward FLOPs of every drawn sequence (2 FLOP per multiply-add)
    d, F, Q = mc.d_model, mc.d_ff, mc.codebook_size
    fwd = B * mc.n_layers * ((6 * d * d + 4 * d * F + 2 * Q * d + 2 * d * d)
                             * N + 2 * N * (N + 1) * d)
    print(json.dumps({
        "metric": "direct autoregressive samples/sec (chain rule), 1 MI355X",
        "value": B / (ms / 1e3), "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": mc.precision, "data": "synthetic",
        "config": {"workload": f"{mc.L}x{mc.L}, VQ transformer "
                               f"d={mc.d_model} L={mc.n_layers} "
                               f"heads={mc.n_heads} mlp={mc.d_ff} "
                               f"Q={mc.codebook_size}, {B} samples",
                   "batch": B},
        "algorithmic_tflop_per_step": fwd / 1e12,
        "achieved_tflops": fwd / (ms / 1e3) / 1e12,
        "mean_logpsi": float(out["logpsi"].mean().item()),
        "kernels": per_kernel}))


def bench_vmc(args, vq, torch, np, mc, make_params):
    """One VMC step of the whole batch (direct samples, their local energies
    in the dedup form, the energy gradient of eq. (3) through the
    straight-through estimator, an Adam update of the parameters), every
    stage on the device; fresh uniform numbers per step.  One JSON line."""
    B, N = mc.batch, mc.N
    dev = torch.device("cuda:0")
    theta = make_params(mc)
    dt_param = torch.float64 if mc.precision == "f64" else torch.float32
    p = torch.tensor(theta, dtype=dt_param, device=dev)
    opt = torch.zeros((2, p.numel()), dtype=dt_param, device=dev)
    cfg = vq.make_config(mc)
    gen = torch.Generator().manual_seed(11)
    us = [torch.rand((B, N), dtype=torch.float64, generator=gen).to(dev)
          for _ in range(args.warmup + args.steps)]
    need = vq.workspace_size(cfg, B, vq.WS_VMC, 0)
    ws = torch.empty(min(need, int(args.ws_gb * (1 << 30))),
                     dtype=torch.uint8, device=dev)
    out = {"spins": torch.empty((B, N), dtype=torch.int8, device=dev),
           "eloc": torch.empty(B, dtype=torch.float64, device=dev),
           "stats": torch.empty(2, dtype=torch.float64, device=dev)}
    energies = []
    k = 0
    for _ in range(args.warmup):
        k += 1
        vq.vmc_step(cfg, p, us[k - 1], 1e-3, opt, step=k, ws=ws, check=False,
                    out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    vq.profile_reset()
    vq.profile_enable(True)
    e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    e0.record(stream)
    for _ in range(args.steps):
        k += 1
        vq.vmc_step(cfg, p, us[k - 1], 1e-3, opt, step=k, ws=ws, check=False,
                    out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    vq.profile_enable(False)
    ms = e0.elapsed_time(e1) / args.steps
    prof = vq.profile_read()
    vq.api._check_status(ws)
    per_kernel = {k2: {"ms_per_step": v[0] / args.steps,
                       "launches_per_step": v[1] / args.steps}
                  for k2, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    st = out["stats"].cpu().numpy().tolist()
    print(json.dumps({
        "metric": "VMC steps/sec (direct samples, dedup local energy, "
                  "straight-through energy gradient, Adam), 1 MI355X",
        "value": 1e3 / ms, "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "samples_per_s": B / (ms / 1e3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": mc.precision, "data": "synthetic",
        "config": {"workload": f"{mc.L}x{mc.L}, VQ transformer "
                               f"d={mc.d_model} L={mc.n_layers} "
                               f"heads={mc.n_heads} mlp={mc.d_ff} "
                               f"Q={mc.codebook_size}, {B} samples per step",
                   "batch": B},
        "last_step_energy": {"mean": st[0], "variance": st[1]},
        "kernels": per_kernel}))


def bench_sweep(args, vq, torch, np, mc, make_params, make_spins):
    """Redundancy sweep: every codebook scaled by alpha (a larger codebook
    scale makes the codes less sensitive to a changed input), dedup with and
    without certified code reuse against plain, on the same spins.  Reports
    the changed rows per layer, the certified fraction and the speed-up per
    alpha; one JSON line."""
    from workloads import scale_codebooks
    B = mc.batch
    dev = torch.device("cuda:0")
    theta = make_params(mc)
    spins = make_spins(mc)
    sp = torch.tensor(spins, device=dev)
    ws_cap = int(args.ws_gb * (1 << 30))
    out = {"eloc": torch.empty(B, dtype=torch.float64, device=dev),
           "counters": torch.empty(vq.NCOUNTERS, dtype=torch.int64,
                                   device=dev)}
    cfg0 = vq.make_config(mc)
    need = max(vq.workspace_size(cfg0, B, vq.DEDUP, 0),
               vq.workspace_size(cfg0, B, vq.PLAIN, 0))
    ws = torch.empty(min(need, ws_cap), dtype=torch.uint8, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    p1 = torch.tensor(theta, dtype=torch.float32, device=dev)
    if not args.no_autotune:
        vq.autotune(cfg0, p1, sp[:min(B, 512)], vq.DEDUP, ws=ws)

    def timed(cfg, p, mode):
        vq.local_energy(cfg, p, sp, mode, stats=False, counters=True, ws=ws,
                        check=False, out=out)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record(stream)
        for _ in range(args.steps):
            vq.local_energy(cfg, p, sp, mode, stats=False, counters=True,
                            ws=ws, check=False, out=out)
        b.record(stream)
        torch.cuda.synchronize()
        return (a.elapsed_time(b) / args.steps,
                counters_dict(vq, out["counters"].cpu().numpy(),
                              mc.n_layers))

    rows = []
    for alpha in (0.5, 1.0, 2.0, 4.0, 8.0):
        p = torch.tensor(scale_codebooks(mc, theta, alpha),
                         dtype=torch.float32, device=dev)
        ms_p, _ = timed(vq.make_config(mc), p, vq.PLAIN)
        entry = {"alpha": alpha, "plain_ms": ms_p,
                 "plain_evals_per_s": B / (ms_p / 1e3)}
        for flags in (0, vq.FLAG_CERTIFIED_VQ):
            ms, ctr = timed(vq.make_config(mc, flags=flags), p, vq.DEDUP)
            nb = max(ctr["neighbours"], 1)
            searched = ctr["vq_rows"] + ctr["vq_certified"]
            entry[f"dedup_flags{flags}"] = {
                "ms": ms, "evals_per_s": B / (ms / 1e3),
                "speedup_vs_plain": ms_p / ms,
                "changed_rows_per_neighbour": [c / nb for c in ctr["changed"]],
                "certified_fraction": (ctr["vq_certified"] / searched
                                       if searched else 0.0)}
        entry["u_over_N_last_layer"] = (
            entry["dedup_flags0"]["changed_rows_per_neighbour"][-1] / mc.N)
        rows.append(entry)
        print(f"sweep alpha={alpha}: plain {ms_p:.0f} ms, dedup "
              f"{entry['dedup_flags0']['ms']:.0f} ms", file=sys.stderr,
              flush=True)
        del p
    print(json.dumps({
        "metric": "redundancy sweep: dedup vs plain local-energy evals/sec "
                  "against the codebook scale alpha, 1 MI355X",
        "config": {"workload": f"{mc.L}x{mc.L} periodic Heisenberg, "
                               f"d={mc.d_model} L={mc.n_layers} "
                               f"Q={mc.codebook_size}, {B} seeded Sz=0 "
                               "samples, codebooks scaled by alpha",
                   "batch": B, "steps": args.steps},
        "dtype": mc.precision, "data": "synthetic", "sweep": rows}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="large")
    ap.add_argument("--workload", default="eloc",
                    choices=["eloc", "grad", "multi", "sweep", "sample",
                             "vmc"],
                    help="eloc: local energy (default); grad: weighted "
                         "straight-through gradient of the 20x20 workload; "
                         "multi: mixed-lattice batch in one call; sweep: "
                         "codebook-scale redundancy sweep; sample: direct "
                         "autoregressive sampling; vmc: one VMC step")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--flags", type=int, default=0,
                    help="1 = certified VQ code reuse")
    ap.add_argument("--ws-gb", type=float, default=192.0,
                    help="workspace cap in GiB (of 288 GB HBM; larger chunks "
                         "mean fewer, fuller launches)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch choices instead of timing "
                         "the variants on the first 512 samples")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON file of launch choices: read them from it "
                         "when present for this device and model width, "
                         "else time them and store them there")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the steps, copy a buffer of this many MiB "
                         "once (a kernel of known traffic that calibrates "
                         "hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only: the "
                          "local energy of each sample is independent, so "
                          "several GPUs would split the batch; run with "
                          "--gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import paper_2212_11296_amd as vq
    from workloads import config_by_name, make_params, make_spins, with_batch

    if args.workload == "multi":
        bench_multi(args, vq, torch, np, make_params, make_spins, with_batch)
        return
    if args.workload == "grad":
        mc = config_by_name("grad")
        if args.batch:
            mc = with_batch(mc, args.batch)
        bench_grad(args, vq, torch, np, mc, make_params, make_spins)
        return
    mc = config_by_name(args.config)
    if args.batch:
        mc = with_batch(mc, args.batch)
    if args.workload == "sweep":
        bench_sweep(args, vq, torch, np, mc, make_params, make_spins)
        return
    if args.workload == "sample":
        bench_sample(args, vq, torch, np, mc, make_params)
        return
    if args.workload == "vmc":
        bench_vmc(args, vq, torch, np, mc, make_params)
        return
    B = mc.batch
    dev = torch.device("cuda:0")
    theta = make_params(mc)
    spins = make_spins(mc)
    dt_param = torch.float64 if mc.precision == "f64" else torch.float32
    p = torch.tensor(theta, dtype=dt_param, device=dev)
    sp = torch.tensor(spins, device=dev)
    cfg = vq.make_config(mc, flags=args.flags)
    ws_cap = int(args.ws_gb * (1 << 30))
    need = vq.workspace_size(cfg, B, vq.DEDUP, 0)
    ws = torch.empty(min(need, ws_cap), dtype=torch.uint8, device=dev)
    out = {"eloc": torch.empty(B, dtype=torch.float64, device=dev),
           "stats": torch.empty(2, dtype=torch.float64, device=dev),
           "ratios": torch.empty((B, 2 * mc.N), dtype=torch.float64,
                                 device=dev),
           "counters": torch.empty(vq.NCOUNTERS, dtype=torch.int64,
                                   device=dev)}

    def step(mode, w):
        vq.local_energy(cfg, p, sp, mode, ratios=True, counters=True, ws=w,
                        check=False, out=out)

    exp_rate = None
    if mc.precision == "bf16":
        exp_rate = vq.probe_exp_rate()
    choices = None
    if not args.no_autotune:
        nt = min(B, 512)
        if args.tuning_cache:
            from paper_2212_11296_amd import tuning
            choices, _ = tuning.autotune_cached(cfg, p, sp[:nt],
                                                args.tuning_cache, ws=ws)
        else:
            choices = vq.autotune(cfg, p, sp[:nt], vq.DEDUP, ws=ws)

    if args.copy_probe_mib > 0:
        n_el = args.copy_probe_mib << 18
        src = torch.ones(n_el, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(vq.DEDUP, ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    vq.profile_reset()
    vq.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step(vq.DEDUP, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    vq.profile_enable(False)
    ms = e0.elapsed_time(e1) / args.steps
    prof = vq.profile_read()
    ctr_d = counters_dict(vq, out["counters"].cpu().numpy(), mc.n_layers)
    stats = out["stats"].cpu().numpy().tolist()
    ratios0 = out["ratios"][0].cpu().numpy()
    parity = golden_parity(mc, out)
    vq.load_library()
    st = vq.api._check_status(ws)
    value = B / (ms / 1000.0)

    flops = flops_model(mc, ctr_d, B)
    per_kernel = {k: {"ms_per_step": v[0] / args.steps,
                      "launches_per_step": v[1] / args.steps}
                  for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}
    dom = next(iter(per_kernel))
    dom_total_ms = prof[dom][0]
    dom_launches = prof[dom][1]
    mpeak = PEAK["bf16"] if mc.precision == "bf16" else PEAK["fp32"]
    if dom in flops and dom_total_ms > 0:
        flop_per_launch = flops[dom] * args.steps / dom_launches
        avg_ms = dom_total_ms / dom_launches
        achieved = flop_per_launch / (avg_ms / 1e3) / 1e12
        roof = {"bound": "mfma", "kernel": dom, "achieved": achieved,
                "peak": mpeak, "unit": "TFLOP/s", "frac": achieved / mpeak,
                "traffic": measured_traffic(dom, mc,
                                            round(dom_launches / args.steps)),
                "flop_per_launch": flop_per_launch,
                "avg_launch_ms": avg_ms,
                "launches_per_step": dom_launches / args.steps}
        if dom.startswith("attention") and exp_rate:
            pk = 4.0 * mc.d_head * exp_rate / 1e12
            roof["exp_bound"] = {
                "exps_per_s": exp_rate, "peak": pk, "unit": "TFLOP/s",
                "frac": achieved / pk,
                "what": "one exponential per (query, key) pair at the "
                        "measured v_exp_f32 issue rate"}
    else:
        roof = {"bound": None, "kernel": dom, "achieved": None, "peak": None,
                "unit": None, "frac": None, "traffic": None}
    # matrix-core phases: algorithmic FLOP/s against the dense peak
    util = {}
    for k in ("qkv", "mlp", "vq"):
        if k in prof and prof[k][0] > 0:
            ach = flops[k] * args.steps / (prof[k][0] / 1e3) / 1e12
            util[k] = {"achieved": ach, "frac": ach / mpeak,
                       "ms_per_step": prof[k][0] / args.steps}

    plain = None
    if not args.no_plain and args.plain_steps > 0:
        need_p = vq.workspace_size(cfg, B, vq.PLAIN, 0)
        del ws
        torch.cuda.empty_cache()
        wsp = torch.empty(min(need_p, ws_cap), dtype=torch.uint8, device=dev)
        step(vq.PLAIN, wsp)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.plain_steps):
            step(vq.PLAIN, wsp)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_p = e0.elapsed_time(e1) / args.plain_steps
        ctr_p = counters_dict(vq, out["counters"].cpu().numpy(), mc.n_layers)
        fl_p = flops_model(mc, ctr_p, B)
        plain = {"value": B / (ms_p / 1000.0), "ms_per_step": ms_p,
                 "steps": args.plain_steps,
                 "algorithmic_tflop_per_step": sum(fl_p.values()) / 1e12,
                 "max_abs_diff_mean_energy_vs_dedup":
                     abs(out["stats"].cpu().numpy()[0] - stats[0])}
        del wsp

    cpu = None
    spot_err = None
    if not args.no_cpu_baseline:
        n_nb0 = int(np.count_nonzero(ratios0))
        cpu, spot_err = cpu_baseline(mc, theta, spins, ratios0, n_nb0,
                                     args.cpu_seconds)
        if "dedup" in cpu:
            e0 = float(out["eloc"][0].item())
            cpu["dedup"]["gpu_eloc_rel_err"] = abs(e0 - cpu["dedup"]["eloc"]) / \
                abs(cpu["dedup"]["eloc"])

    res = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": mc.precision, "data": "synthetic",
        "config": {"workload": (
                       (f"{mc.N}-site {'periodic' if mc.periodic else 'open'} "
                        f"transverse-field Ising chain (Gamma={mc.gamma})"
                        if mc.hamiltonian == "tfim" else
                        f"{mc.L}x{mc.L} "
                        f"{'periodic' if mc.periodic else 'open'} Heisenberg")
                       + (f", tokens of {mc.group} spins ({mc.T} positions)"
                          if mc.group > 1 else "")
                       + (", bidirectional encoder (mean-pooled log psi)"
                          if mc.encoder else "")
                       + f", VQ transformer d={mc.d_model} L={mc.n_layers}"
                       + (" + attention-only half-block" if mc.attn_tail
                          else "") + " "
                       f"heads={mc.n_heads} mlp={mc.d_ff} "
                       f"Q={mc.codebook_size}x{mc.vq_heads}, {B} seeded "
                       + ("uniform" if mc.hamiltonian == "tfim" else "Sz=0")
                       + " samples, dedup local energy"),
                   "L": mc.L, "batch": B, "mode": "dedup",
                   "flags": args.flags, "precision": mc.precision},
        "roofline": roof,
        "mfma_utilisation": util,
        "cpu_baseline": cpu,
        "oracle_parity": parity,
        "plain": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "algorithmic_tflop_per_step": sum(flops.values()) / 1e12,
        "achieved_tflops_overall": sum(flops.values()) / (ms / 1e3) / 1e12,
        "mean_energy": stats[0], "energy_variance": stats[1],
        "oracle_spot_rel_err_ratio": spot_err,
        "tuning": (None if choices is None else
                   {"qkv_mb": choices[0], "mlp_mb": choices[1],
                    "vq_mb": choices[2]}),
        "counters_per_step": ctr_d,
        "kernels": per_kernel,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
