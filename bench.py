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
# Attention at head width 16-32 is bound by the vector unit, not by the
# algorithmic matrix-core work: every (query, key) pair needs one
# exponential, and v_exp_f32 issues at half the rate of plain FP32 VALU
# instructions on gfx950 (8 lanes per SIMD per cycle; a timing probe of
# independent exponential chains gives 7.47 lane-ops per SIMD-cycle against
# 14.7 for additions).  256 CUs x 4 SIMDs x 8 x 2.4 GHz = 1.97e13
# exponentials per second bound the pair rate; the attention peak is that
# rate times the algorithmic FLOPs of a pair (4 d_head: q.k and p.v).
EXP_RATE = 256 * 4 * 8 * 2.4e9
TRAFFIC_FILE = "profiles/attention_dedup_16x16_bf16__hbm_traffic.json"


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
    P = onet.unpack(mc, theta)
    bl = lattice.bonds(mc.L, mc.periodic)
    nb = lattice.neighbours(spins[0], bl)
    seqs = [spins[0]]
    t0 = time.perf_counter()
    lp0 = onet.forward(mc, P, spins[0:1])["logpsi"][0]
    per = time.perf_counter() - t0
    k = int(max(4, min(len(nb), budget_s / max(per, 1e-3))))
    t0 = time.perf_counter()
    sub = np.stack([lattice.swap(spins[0], p1, p2) for _, p1, p2 in nb[:k]])
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
    return {"value": rate, "unit": UNIT, "cores": cores, "kind": "oracle",
            "sample": (f"sample 0 of the batch: log psi of the sample and of "
                       f"its first {k} of {len(nb)} exchange neighbours, "
                       f"NumPy float64, {dt:.1f} s; rate scaled by "
                       f"1 + n_neighbours evaluations per local energy")
            }, err


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
            bound, peak = "alu", 4.0 * mc.d_head * EXP_RATE / 1e12
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


def bench_multi(args, vq, torch, np, make_params, make_spins):
    """Mixed-lattice batch (6x6 .. 20x20, one model each, 512 .. 8192
    samples): one vqnqs_local_energy_multi call per step, replayed as a
    captured graph, against one vqnqs_local_energy call per lattice."""
    from workloads import MULTI_LATTICE
    dev = torch.device("cuda:0")
    jobs = []
    for mc in MULTI_LATTICE:
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
                               "512/1024/2048/4096/8192 seeded Sz=0 samples, "
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="large")
    ap.add_argument("--workload", default="eloc",
                    choices=["eloc", "grad", "multi"],
                    help="eloc: local energy (default); grad: weighted "
                         "straight-through gradient of the 20x20 workload; "
                         "multi: mixed-lattice batch in one call")
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
        bench_multi(args, vq, torch, np, make_params, make_spins)
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

    choices = None
    if not args.no_autotune:
        nt = min(B, 512)
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
    if dom in flops and dom_total_ms > 0:
        flop_per_launch = flops[dom] * args.steps / dom_launches
        avg_ms = dom_total_ms / dom_launches
        achieved = flop_per_launch / (avg_ms / 1e3) / 1e12
        if dom.startswith("attention"):
            bound, peak = "alu", 4.0 * mc.d_head * EXP_RATE / 1e12
        else:
            bound, peak = "mfma", PEAK["bf16"]
        roof = {"bound": bound, "kernel": dom, "achieved": achieved,
                "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(dom, mc,
                                            round(dom_launches / args.steps)),
                "flop_per_launch": flop_per_launch,
                "avg_launch_ms": avg_ms}
    else:
        roof = {"bound": None, "kernel": dom, "achieved": None, "peak": None,
                "unit": None, "frac": None, "traffic": None}

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

    res = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": mc.precision, "data": "synthetic",
        "config": {"workload": (f"{mc.L}x{mc.L} periodic Heisenberg, VQ "
                                f"transformer d={mc.d_model} L={mc.n_layers} "
                                f"heads={mc.n_heads} mlp={mc.d_ff} "
                                f"Q={mc.codebook_size}, {B} seeded Sz=0 "
                                f"samples, dedup local energy"),
                   "L": mc.L, "batch": B, "mode": "dedup",
                   "flags": args.flags, "precision": mc.precision},
        "roofline": roof,
        "cpu_baseline": cpu,
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
