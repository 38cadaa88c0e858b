"""Benchmark of the primal-dual Gibbs sweep on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Workload (seeded, synthetic): the plain grid -- 1024 x 1024 open 4-neighbour
grid, q = 4, log-tables N(0, 0.2) per edge, log-unaries N(0, 1), FP32 tables,
64 independent chains, sampler seed 0.  A step is one full sweep: the dual
phase over every edge and chain, then the primal phase over every node and
chain (with marginal counting).  The metric is chain * (|V| + |E|) updates/s
with every input resident in HBM.

Prints one JSON line.  ``roofline`` describes the dominant kernel (the dual
phase): it is bound by integer VALU work (Philox draws), so achieved and peak
are VALU issue slots per second; ``cpu_baseline`` is the FP64 oracle timed on
the host cores on one step of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ---- VALU roofline of the dual kernel ---------------------------------------
# Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 full-rate 32-bit VALU
# lane-operations per second.  Algorithmic work of one dual draw, in full-rate
# issue slots: one fifth of a Philox4x32-10 call -- 10 rounds, each two 32x32->64
# multiplies (v_mad_u64_u32, measured full rate on gfx950) and two three-input
# xors (v_bitop3_b32) -- plus three compares that decide the draw (11 slots).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
PHILOX_SLOTS = 10 * (2 + 2)
DRAW_SLOTS = PHILOX_SLOTS / 5.0 + 3.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--chains", type=int, default=64)
    p.add_argument("--side", type=int, default=1024)
    p.add_argument("--no-cpu-baseline", action="store_true")
    return p.parse_args()


def cpu_baseline(model, C, seed):
    from oracle import oracle
    dec = oracle.decompose(model)
    uid = np.arange(1, model.m + 1, dtype=np.uint64)
    x = oracle.init_state(model, C, seed)
    t0 = time.perf_counter()
    oracle.run(model, dec, uid, seed, x, 0, 1, burn_in=0)
    dt = time.perf_counter() - t0
    return {"value": C * (model.n + model.m) / dt, "unit": "updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"1 sweep of the full workload, {C} chains, {dt:.2f} s wall"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sampler's "
              "chains would shard across GPUs with no per-sweep communication, but no "
              "multi-GPU run is part of this build.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1611_06684_amd import workloads as W
    from paper_1611_06684_amd.pdg import Sampler

    side, C, seed = args.side, args.chains, 0
    model = W.table_grid(side, side, 4, seed=0)
    s = Sampler(model, C, seed=seed, burn_in=0)
    s.init()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        s.dual_phase()
        s.primal_phase()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        s.dual_phase()
        ev[k][1].record(stream)
        s.primal_phase()
        ev[k][2].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    dual_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    primal_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    s.sync()

    updates = C * (model.n + model.m)
    value = updates * args.steps / (total_ms / 1e3)
    draws_per_launch = model.m * 9 * C
    achieved = draws_per_launch * DRAW_SLOTS / (dual_ms / 1e3)
    out = {
        "metric": "chain*(|V|+|E|) updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain grid {side}x{side}, q=4, FP32 tables, {C} chains",
                   "nodes": model.n, "edges": model.m, "chains": C, "seed": seed,
                   "dual_ms": dual_ms, "primal_ms": primal_ms, "wall_s": wall},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_LANE_OPS,
                     "unit": "VALU lane-ops/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": None, "kernel": "k_dual<4,64>",
                     "work_per_draw_slots": DRAW_SLOTS},
    }
    s.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(model, C, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
