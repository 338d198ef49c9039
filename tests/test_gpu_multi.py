"""Multi-lattice batched launch, HIP-graph replay and the autotuner.

* A mixed batch (several lattices, precisions and models in one call)
  gives, bit for bit, the results of one local-energy call per lattice:
  sequentially, on concurrent internal streams, and replayed as a captured
  graph.  The graph is replayed several times with the program's own eager
  work and synchronisations in between, with the outputs cleared before
  every replay, and every replay is checked.
* A workspace smaller than the whole batch (chunked jobs) changes nothing.
* A bad spin in any job shows in the call's status word.
* Launch choices (rows per wave, including four rows per wave in the
  codebook search) never change results; the autotuner picks valid ones.
"""
import numpy as np
import pytest
import torch

import paper_2212_11296_amd as vq
from workloads import (CONFIGS, MULTI_LATTICE, make_params, make_spins,
                       with_batch)

from gpu_common import dev_params, dev_spins, host, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def _jobs():
    mcs = [with_batch(CONFIGS["small"], 24),
           with_batch(MULTI_LATTICE[0], 40),            # 6x6 BF16
           with_batch(MULTI_LATTICE[1], 16),            # 8x8 BF16
           with_batch(CONFIGS["medium"], 8)]            # 10x10 FP32
    jobs = []
    for mc in mcs:
        jobs.append((vq.make_config(mc), dev_params(make_params(mc),
                                                    mc.precision),
                     dev_spins(make_spins(mc))))
    return mcs, jobs


def _singles(jobs):
    return [vq.local_energy(cfg, p, s, vq.DEDUP, ratios=True)
            for cfg, p, s in jobs]


def _same(outs, ref):
    for o, r in zip(outs, ref):
        assert np.array_equal(host(o["eloc"]), host(r["eloc"]))
        assert np.array_equal(host(o["ratios"]), host(r["ratios"]))
        assert np.array_equal(host(o["stats"]), host(r["stats"]))


@pytest.mark.parametrize("flags", [0, vq.MULTI_CONCURRENT])
def test_multi_equals_single_calls(flags):
    say(f"multi eager flags={flags}")
    mcs, jobs = _jobs()
    ref = _singles(jobs)
    outs = vq.local_energy_multi(jobs, flags=flags, ratios=True)
    _same(outs, ref)


def test_multi_graph_replays():
    say("multi graph replays")
    mcs, jobs = _jobs()
    ref = _singles(jobs)
    ws = torch.empty(vq.workspace_size_multi(jobs), dtype=torch.uint8,
                     device="cuda")
    flags = vq.MULTI_CONCURRENT | vq.MULTI_GRAPH
    outs = vq.local_energy_multi(jobs, flags=flags, ratios=True, ws=ws)
    _same(outs, ref)
    for rep in range(3):
        for o in outs:
            for t in o.values():
                t.zero_()
        # eager work of the program between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * x).sum().item()
        cfg, p, s = jobs[rep % len(jobs)]
        vq.local_energy(cfg, p, s, vq.DEDUP)
        torch.cuda.synchronize()
        vq.local_energy_multi(jobs, flags=flags, ratios=True, ws=ws, outs=outs)
        torch.cuda.synchronize()
        _same(outs, ref)


def test_multi_small_workspace_chunks_jobs():
    say("multi chunked")
    mcs, jobs = _jobs()
    ref = _singles(jobs)
    need = vq.workspace_size_multi(jobs)
    ws = torch.empty(need // 3, dtype=torch.uint8, device="cuda")
    outs = vq.local_energy_multi(jobs, flags=vq.MULTI_CONCURRENT, ratios=True,
                                 ws=ws)
    _same(outs, ref)


def test_multi_bad_spin_reported():
    mcs, jobs = _jobs()
    cfg, p, s = jobs[0]
    bad = s.clone()
    bad[3, 5] = 0
    jobs[0] = (cfg, p, bad)
    with pytest.raises(vq.VQNQSError) as e:
        vq.local_energy_multi(jobs, flags=vq.MULTI_CONCURRENT)
    assert e.value.status == 6


@pytest.mark.parametrize("mc", [with_batch(MULTI_LATTICE[1], 48),
                                with_batch(CONFIGS["large"], 6)],
                         ids=["8x8_d128", "16x16_d128"])
def test_launch_choices_do_not_change_results(mc):
    say(f"tuning invariance {mc.name}")
    cfg = vq.make_config(mc)
    p, s = dev_params(make_params(mc), "bf16"), dev_spins(make_spins(mc))
    outs = []
    for ch in ([1, 1, 1], [2, 2, 2], [1, 2, 1], [2, 1, 2], [1, 1, 4],
               [2, 2, 4]):
        vq.set_tuning(cfg, ch)
        o = vq.local_energy(cfg, p, s, vq.DEDUP, ratios=True)
        outs.append((host(o["eloc"]), host(o["ratios"])))
    for e, r in outs[1:]:
        assert np.array_equal(e, outs[0][0])
        assert np.array_equal(r, outs[0][1])
    ch = vq.autotune(cfg, p, s)
    assert ch[0] in (1, 2) and ch[1] in (1, 2) and ch[2] in (1, 2, 4)
    o = vq.local_energy(cfg, p, s, vq.DEDUP, ratios=True)
    assert np.array_equal(host(o["eloc"]), outs[0][0])
    with pytest.raises(vq.VQNQSError):
        vq.set_tuning(cfg, [3, 1, 1])
