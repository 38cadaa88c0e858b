"""Benchmark of the primal-dual Gibbs sweep on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--workload dynamic-sparse|plain-grid|tiny|batched|learned]

Workloads (seeded, synthetic; recipes in workloads.py):
  dynamic-sparse (default, the headline line: the largest single-GPU
    configuration): Chung-Lu power-law graph, 2^22 nodes, exponent 2.5, mean
    degree 8, q = 8, log-tables N(0, 0.15), log-unaries N(0, 1), FP32 tables,
    32 chains; every 10 sweeps 1 % of the live edges are removed and as many
    inserted (edit batches prepared on the device before timing; the edits
    themselves are timed).
  plain-grid: 1024 x 1024 open 4-neighbour grid, q = 4, log-tables N(0, 0.2)
    per edge, log-unaries N(0, 1), FP32 tables, 64 independent chains.
  tiny: 4 x 4 binary grid (Ising tables exp(J s s'), J ~ U(-0.3, 0.3), unaries
    exp(h s), h ~ N(0, 0.5)), FP64, one chain: bound by latency, so its line is
    sweeps/s (steps = sweeps, run in batches of one launch each).
  batched: 4096 independent graphs: 4032 sparse graphs with N ~ logU[100, 50000],
    mean degree U{3..12}, q ~ U{2,3,5}, plus 64 complete binary graphs on 2048
    nodes (Ising tables, J ~ N(0, 0.5 / sqrt(2048))); 8 chains.  Built directly
    as one context per state count, each tuned by pdg_tune; the timed sweeps
    are replays of one captured HIP graph of --graph-sweeps sweeps of every
    context.  After the timed region, the dense graphs' gather is timed in its
    vector and FP64 matrix-core forms (config.dense_gather).
  learned: the learned block proposal on a 512 x 512 binary grid (8 x 8
    blocks, 128 chains): the proposal network is trained on plain-sampler
    block states, then ESS/s of (learned step + plain sweep) is compared with
    plain sweeps at equal marginal error; steps = iterations.
A step is one full sweep: the dual phase over every edge and chain, then the
primal phase over every node and chain (with marginal counting).  The metric is
chain * (|V| + |E|) updates/s with every input resident in HBM.

Prints one JSON line.  ``roofline`` describes the dominant kernel, the dual:
it is bound by integer ALU work (Philox draws and their decision logic), so
achieved and peak are full-rate 32-bit lane-operation slots per second.  ``roofline_primal`` puts the primal phase against the
HBM roof (algorithmic bytes: the h records and dual words of every incidence,
per node its base row, state and counters).  ``traffic`` (HBM bytes per launch
from rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a plain copy) is read from the
summary under profiles/ and is null when that summary was taken from other
kernel sources than the ones built now.  ``cpu_baseline`` is the FP64 oracle
timed on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ---- VALU roofline of the dual kernel ---------------------------------------
# Peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6e12 full-rate 32-bit VALU
# lane-operations per second (the chip's 157.3 TFLOP/s FP32 vector rate counts
# an FMA as two).  Algorithmic work of one dual draw, in those slots: one fifth
# of a Philox4x32-10 call plus the three compares that decide the draw.  A call
# is 10 rounds of two 32x32->64 multiplies (v_mad_u64_u32, not a full-rate op)
# and two three-input xors; its cost is the measured one, 78.3 slots (the chip
# runs 1.00e12 calls/s with every lane busy: profiles/valu_rates.txt), so a
# draw is 78.3 / 5 + 3 = 18.7 slots.
PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9
PHILOX_SLOTS = 78.3
DRAW_SLOTS = PHILOX_SLOTS / 5.0 + 3.0
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
# what the path computes in (FP32-table workloads): FP64 decomposition and field
# sums, FP32 exp in the node draw, 24-bit integer uniforms and thresholds
DTYPE = "f64 fields + f32 exp + u32 draws"
KERNEL_SOURCES = ["pdg_kernels.hpp", "pdg_rng.hpp", "pdg_store.hpp", "pdg.hip"]


def kernel_digest():
    """First 16 hex digits of the sha256 of the HIP sources the kernels are
    built from (a profile summary records the digest it was taken with)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_06684_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_traffic(summary, label):
    """HBM bytes per launch recorded under `label` in profiles/<summary>, as a line
    ``traffic <label> <bytes> sources <digest>``; None when absent or taken from
    other kernel sources."""
    try:
        text = open(os.path.join(PROFILES, summary)).read()
    except OSError:
        return None
    for line in text.splitlines():
        f = line.split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == label and f[3] == "sources":
            return float(f[2]) if f[4] == kernel_digest() else None
    return None


def host_info():
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def chain_major(model, C):
    """Whether the context keeps its dual words chain-major (one 64-bit word per
    chain and record): 17..32 chains with q_max >= 6."""
    return model.q_max >= 6 and 17 <= C <= 32


def record_words(model, C, D):
    """Bytes of dual words per incidence record with D entries: chain-major 8 C;
    otherwise one chain mask per entry, 4 D bytes (C <= 32) or 8 D per block of
    64 chains."""
    if chain_major(model, C):
        return 8 * C
    return 4 * D if C <= 32 else 8 * D * ((C + 63) // 64)


def primal_bytes(model, C):
    """Algorithmic HBM bytes of one primal phase: per incidence the record's h
    (8 D bytes, FP64) and its dual words (record_words), D = (q_node - 1)
    (q_other - 1); per node its base row (8 q_max), new states (C), counters
    read and written (8 q_max) and segment offset and count (8)."""
    D = (model.q[model.src].astype(np.int64) - 1) * (model.q[model.dst] - 1)
    qm = model.q_max
    return int(2 * (8 * D + record_words(model, C, D)).sum() + model.n * (16 * qm + C + 8))


def dual_bytes(model, C):
    """Algorithmic HBM bytes of one dual phase: per edge with D =
    (q_src-1)(q_dst-1) entries, slot metadata (uid 8, src 4, dst 4, record
    positions 8), the sign word (8) and D threshold pairs (8 D), the endpoint
    states (2 C bytes) and the dual words written to each of the two records
    (record_words)."""
    D = (model.q[model.src].astype(np.int64) - 1) * (model.q[model.dst] - 1)
    return int((32 + 2 * C + 8 * D + 2 * record_words(model, C, D)).sum())


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--warmup", type=int, default=None)
    p.add_argument("--workload", choices=["dynamic-sparse", "plain-grid", "tiny", "batched",
                                          "learned"],
                   default="dynamic-sparse")
    p.add_argument("--epochs", type=int, default=2, help="learned workload: training epochs")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--batch-graphs", type=int, default=4096,
                   help="batched workload: number of graphs (1/64 of them dense)")
    p.add_argument("--graph-sweeps", type=int, default=10,
                   help="batched workload: sweeps per captured HIP graph")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="after the run, copy a buffer of this many MiB three times (a plain "
                        "copy kernel of known size, to calibrate memory counters)")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _native_oracle():
    """The oracle built for this host (-O3 -march=native); the portable build
    when no compiler is at hand.  Returns the flags used."""
    from oracle import oracle
    try:
        oracle.use_library(oracle.build_native())
        return " ".join(oracle.FLAGS_NATIVE)
    except (OSError, subprocess.CalledProcessError) as e:
        log(f"native oracle build failed ({e}); timing the portable build")
        oracle.use_library(None)
        return " ".join(oracle.FLAGS)


def cpu_baseline(model, C, seed, what="1 sweep of the full workload", sweeps=1):
    """The oracle, as it stands, on `sweeps` sweeps of `model` with C chains."""
    from oracle import oracle
    flags = _native_oracle()
    dec = oracle.decompose(model)
    uid = np.arange(1, model.m + 1, dtype=np.uint64)
    x = oracle.init_state(model, C, seed)
    t0 = time.perf_counter()
    oracle.run(model, dec, uid, seed, x, 0, sweeps, burn_in=0)
    dt = time.perf_counter() - t0
    return {"value": C * (model.n + model.m) * sweeps / dt, "unit": "updates/s",
            "cores": min(oracle.num_threads(), C), "kind": "oracle",
            "sample": f"{what}, {C} chains, {dt:.2f} s wall",
            "compile": flags, "host": host_info()}


def timed_sweeps(s, steps, stream, between=None):
    """Times `steps` sweeps on `stream` with events around each phase; `between(k)`
    runs before sweep k (edits)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for k in range(steps):
        if between is not None:
            between(k)
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
    return total_ms, dual_ms, primal_ms, wall


def time_log_v(s, stream, reps=20):
    """Average time of one partition-function estimate (log V of every chain,
    between the phases of a sweep); outside the timed sweeps."""
    import torch
    ms = 0.0
    for _ in range(reps):
        s.dual_phase()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.log_v()
        b.record(stream)
        s.primal_phase()
        b.synchronize()
        ms += a.elapsed_time(b)
    return ms / reps


def run_plain(args):
    import torch
    from paper_1611_06684_amd import workloads as W
    from paper_1611_06684_amd.pdg import Sampler
    steps = 200 if args.steps is None else args.steps
    warmup = 20 if args.warmup is None else args.warmup
    side, C, seed = 1024, 64, 0
    model = W.table_grid(side, side, 4, seed=0)
    s = Sampler(model, C, seed=seed, burn_in=0)
    s.init()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        s.dual_phase()
        s.primal_phase()
    total_ms, dual_ms, primal_ms, wall = timed_sweeps(s, steps, stream)
    log_v_ms = time_log_v(s, stream)
    s.sync()
    s.close()
    updates = C * (model.n + model.m)
    draws_per_launch = model.m * 9 * C
    achieved = draws_per_launch * DRAW_SLOTS / (dual_ms / 1e3)
    pbytes = primal_bytes(model, C)
    p_gbs = pbytes / (primal_ms / 1e3) / 1e9
    out = {
        "metric": "chain*(|V|+|E|) updates/s",
        "value": updates * steps / (total_ms / 1e3),
        "unit": "updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": total_ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE, "data": "synthetic",
        "config": {"workload": f"plain grid {side}x{side}, q=4, FP32 tables, {C} chains",
                   "nodes": model.n, "edges": model.m, "chains": C, "seed": seed,
                   "dual_ms": dual_ms, "primal_ms": primal_ms, "wall_s": wall,
                   "log_v_ms": log_v_ms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_LANE_OPS,
                     "unit": "VALU lane-ops/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": profile_traffic("plain_grid_sweep_kernels.txt",
                                                "k_dual64<4,true,4>"),
                     "kernel": "k_dual64<4,true,4>",
                     "work_per_draw_slots": DRAW_SLOTS},
        "roofline_primal": {"bound": "hbm", "achieved": p_gbs, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": p_gbs / HBM_PEAK_GBS,
                            "traffic": profile_traffic("plain_grid_sweep_kernels.txt",
                                                       "primal_phase"),
                            "kernel": "k_primal64<4,true,false>", "algorithmic_bytes": pbytes},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(model, C, seed, "2 sweeps of the full workload", sweeps=2)
    return out


def dynamic_cpu_baseline(q, C, seed, every):
    """The oracle on a bounded sample of the dynamic workload: the same recipe at
    2^19 nodes (an eighth of the nodes and edges), one sweep of all C chains, one
    churn step (1 % of the edges removed, as many inserted and decomposed), a
    second sweep on the edited graph; then one sweep with one chain on one core."""
    from oracle import oracle
    from paper_1611_06684_amd import workloads as W
    n = 1 << 19
    flags = _native_oracle()
    model = W.chung_lu(n, q, seed=0)
    dec = oracle.decompose(model)
    churn = W.Churn(n, q, model.meta["weights"], seed=1)
    uid = np.arange(1, model.m + 1, dtype=np.uint64)
    x = oracle.init_state(model, C, seed)
    t0 = time.perf_counter()
    oracle.run(model, dec, uid, seed, x, 0, 1, burn_in=0)
    t_sweep = time.perf_counter() - t0
    t1 = time.perf_counter()
    rem, ns, nd, nL = churn.next_batch(uid)
    keep = ~np.isin(uid, rem)
    cur = W.Model(model.q, model.lam, np.concatenate([model.src[keep], ns]),
                  np.concatenate([model.dst[keep], nd]), np.concatenate([model.Lam[keep], nL]))
    new = oracle.decompose(W.Model(model.q, model.lam, ns, nd, nL))
    dec2 = oracle.Decomposition(np.concatenate([dec.par[keep], new.par]),
                                np.concatenate([dec.rrow[keep], new.rrow]),
                                np.concatenate([dec.rcol[keep], new.rcol]))
    uid2 = np.concatenate([uid[keep], uid[-1] + 1 + np.arange(len(ns), dtype=np.uint64)])
    t_edit = time.perf_counter() - t1
    t2 = time.perf_counter()
    oracle.run(cur, dec2, uid2, seed, x, 1, 1, burn_in=0)
    t_sweep2 = time.perf_counter() - t2
    dt = time.perf_counter() - t0
    ups = C * ((model.n + model.m) + (cur.n + cur.m)) / (t_sweep + t_sweep2 + 2 * t_edit / every)
    threads = min(oracle.num_threads(), C)
    oracle.set_threads(1)
    x1 = np.ascontiguousarray(x[:, :1])
    t3 = time.perf_counter()
    oracle.run(cur, dec2, uid2, seed, x1, 2, 1, burn_in=0)
    t_one = time.perf_counter() - t3
    oracle.set_threads(threads)
    oracle.use_library(None)
    return {"value": ups, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": (f"the dynamic recipe at 2^19 nodes ({model.m} edges): 2 sweeps of {C} "
                       f"chains ({t_sweep:.2f} s, {t_sweep2:.2f} s) around 1 churn step of "
                       f"{len(ns)} removals and insertions ({t_edit:.2f} s, charged as 1/{every} "
                       f"per sweep), {dt:.1f} s wall"),
            "single_core": {"value": (cur.n + cur.m) / t_one, "unit": "updates/s",
                            "sample": f"1 sweep of 1 chain on 1 thread, {t_one:.2f} s"},
            "compile": flags, "host": host_info()}


def run_dynamic(args):
    import torch
    from paper_1611_06684_amd import workloads as W
    from paper_1611_06684_amd import pdg
    from paper_1611_06684_amd.pdg import Sampler
    steps = 50 if args.steps is None else args.steps
    warmup = 10 if args.warmup is None else args.warmup
    n, q, C, seed, every = 1 << 22, 8, 32, 0, 10
    log("building the Chung-Lu graph")
    model = W.chung_lu(n, q, seed=0)
    log(f"graph: {model.n} nodes, {model.m} edges; uploading and decomposing")
    s = Sampler(model, C, seed=seed, burn_in=0, edge_capacity=model.m)
    s.init()
    live = s.uids.clone()
    m_live = int(live.numel())
    # edit batches for every churn point of warmup + timed sweeps, staged on the device
    churn = W.Churn(n, q, model.meta["weights"], seed=1)
    n_batches = (warmup + steps + every - 1) // every
    batches = []
    for _ in range(n_batches):
        pos, bs, bd, bL = churn.next_batch(np.arange(m_live))
        batches.append(tuple(torch.as_tensor(np.ascontiguousarray(a), device="cuda")
                             for a in (pos.astype(np.int64), bs, bd, bL)))
    log(f"{n_batches} edit batches of {len(batches[0][0])} removals + insertions staged")
    state = {"live": live, "b": 0}

    def edit(k):
        if k % every != 0:
            return
        pos, bs, bd, bL = batches[state["b"]]
        state["b"] += 1
        lv = state["live"]
        u = lv[pos].contiguous()
        pdg.pdg_remove_edges(s.ctx, u.numel(), u.data_ptr())
        new = torch.zeros(bs.numel(), dtype=torch.int64, device="cuda")
        pdg.pdg_insert_edges(s.ctx, bs.numel(), bs.data_ptr(), bd.data_ptr(), bL.data_ptr(),
                             new.data_ptr())
        keep = torch.ones(lv.numel(), dtype=torch.bool, device="cuda")
        keep[pos] = False
        state["live"] = torch.cat([lv[keep], new])

    stream = torch.cuda.current_stream()
    for k in range(warmup):
        edit(k)
        s.dual_phase()
        s.primal_phase()
    log("warm-up done")
    total_ms, dual_ms, primal_ms, wall = timed_sweeps(
        s, steps, stream, between=lambda k: edit(warmup + k))
    s.sync()
    s.close()
    del batches
    updates = C * (model.n + m_live)
    draws_per_launch = m_live * 49 * C
    achieved = draws_per_launch * DRAW_SLOTS / (dual_ms / 1e3)
    pbytes = primal_bytes(model, C)
    p_gbs = pbytes / (primal_ms / 1e3) / 1e9
    out = {
        "metric": "chain*(|V|+|E|) updates/s",
        "value": updates * steps / (total_ms / 1e3),
        "unit": "updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": total_ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE, "data": "synthetic",
        "config": {"workload": f"dynamic sparse: Chung-Lu 2^22 nodes, q=8, FP32 tables, {C} chains, "
                               f"1% churn every {every} sweeps",
                   "nodes": model.n, "edges": m_live, "chains": C, "seed": seed,
                   "dual_ms": dual_ms, "primal_ms": primal_ms, "wall_s": wall,
                   "edit_batches_timed": sum(1 for k in range(steps) if (warmup + k) % every == 0),
                   "kernel_sources": kernel_digest()},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_LANE_OPS,
                     "unit": "VALU lane-ops/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": profile_traffic("dynamic_sparse_sweep_kernels.txt",
                                                "k_dual<8,32,true>"),
                     "kernel": "k_dual<8,32,true>", "work_per_draw_slots": DRAW_SLOTS,
                     "units_per_launch": draws_per_launch},
        "roofline_primal": {"bound": "hbm", "achieved": p_gbs, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": p_gbs / HBM_PEAK_GBS,
                            "traffic": profile_traffic("dynamic_sparse_sweep_kernels.txt",
                                                       "primal_phase"),
                            "kernel": "primal phase (k_primal32z + hub pieces + hub finish)",
                            "algorithmic_bytes": pbytes},
    }
    del model
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = dynamic_cpu_baseline(q, C, seed, every)
    return out


def run_tiny(args):
    import torch
    from paper_1611_06684_amd import workloads as W
    from paper_1611_06684_amd.pdg import Sampler
    steps = 100000 if args.steps is None else args.steps
    warmup = 1000 if args.warmup is None else args.warmup
    model = W.ising_grid(4, 4, seed=0)
    C, seed = 1, 0
    s = Sampler(model, C, seed=seed, burn_in=0)
    s.init()
    s.sweep(warmup)
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    a.record(stream)
    s.sweep(steps)
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = a.elapsed_time(b)
    s.close()
    out = {
        "metric": "sweeps/s", "value": steps / (ms / 1e3), "unit": "sweeps/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "tiny: 4x4 binary grid, FP64, 1 chain",
                   "nodes": model.n, "edges": model.m, "chains": C, "seed": seed,
                   "updates_per_s": C * (model.n + model.m) * steps / (ms / 1e3),
                   "wall_s": wall},
        "roofline": {"bound": "latency", "achieved": None, "peak": None, "unit": None,
                     "frac": None, "traffic": None, "kernel": "k_sweeps_lds<2,true,true>"},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle
        dec = oracle.decompose(model)
        x = oracle.init_state(model, C, seed)
        n_cpu = 5000000
        t0 = time.perf_counter()
        oracle.run(model, dec, np.arange(1, model.m + 1, dtype=np.uint64), seed, x, 0, n_cpu, 0)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n_cpu / dt, "unit": "sweeps/s",
                               "cores": min(oracle.num_threads(), C), "kind": "oracle",
                               "sample": f"{n_cpu} sweeps of the same workload, {dt:.2f} s wall"}
    return out


class SamplerGroup:
    """Independent samplers on one stream, swept as one: a phase of the group is
    that phase of every member, in order."""

    def __init__(self, samplers):
        self.samplers = samplers

    def dual_phase(self):
        for s in self.samplers:
            s.dual_phase()

    def primal_phase(self):
        for s in self.samplers:
            s.primal_phase()


FP64_PEAK = 78.6e12


def dense_gather_experiment(sampler, nodes, n_dense, C, stream, reps=20):
    """The dense graphs' gather two ways, outside the timed sweeps: the field of
    state 1 of every node of the complete binary graphs (the first `nodes` nodes
    of the binary context, 2047 incidences each) given the current duals, by
    vector FMAs and by FP64 matrix-core products (pdg_dense_fields).  The
    matrix-core form issues one 16x16x4 product per 4 records of a node, of
    which one column of 16 is used."""
    import torch
    from paper_1611_06684_amd import pdg_block as pb
    ids = torch.arange(nodes, dtype=torch.int32, device=sampler.dev)
    out = torch.empty((nodes, C), dtype=torch.float64, device=sampler.dev)
    sampler.dual_phase()
    ms = {}
    for method, name in ((0, "valu"), (1, "mfma")):
        for _ in range(3):
            pb.pdg_dense_fields(sampler.ctx, nodes, ids.data_ptr(), method, out.data_ptr())
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            pb.pdg_dense_fields(sampler.ctx, nodes, ids.data_ptr(), method, out.data_ptr())
        b.record(stream)
        b.synchronize()
        ms[name] = a.elapsed_time(b) / reps
    sampler.primal_phase()
    recs = n_dense - 1
    useful = 2.0 * nodes * recs * C
    issued = nodes * ((recs + 3) // 4) * (16 * 16 * 4 * 2)
    return {"nodes": nodes, "records_per_node": recs, "chains": C,
            "valu_ms": ms["valu"], "mfma_ms": ms["mfma"],
            "useful_gflop": useful / 1e9, "mfma_issued_gflop": issued / 1e9,
            "mfma_issued_frac_of_fp64_peak": issued / (ms["mfma"] / 1e3) / FP64_PEAK,
            "faster": "valu" if ms["valu"] <= ms["mfma"] else "mfma"}


def run_batched(args):
    """The batched workload at its full recipe: 4096 independent graphs (64 of
    them complete binary graphs on 2048 nodes), one context per state count,
    each tuned by pdg_tune; the timed sweeps are replays of one captured HIP
    graph holding `graph_sweeps` sweeps of every context."""
    import torch
    from paper_1611_06684_amd import pdg
    from paper_1611_06684_amd import workloads as W
    from paper_1611_06684_amd.pdg import Sampler
    K = args.graph_sweeps
    steps = 50 if args.steps is None else args.steps
    steps = max(K, (steps + K - 1) // K * K)
    warmup = 5 if args.warmup is None else args.warmup
    C, seed, n_graphs, n_dense = 8, 0, args.batch_graphs, max(1, args.batch_graphs // 64)
    log(f"building the batch ({n_graphs} graphs, {n_dense} dense) per state count")
    parts = W.batched_by_states(n_graphs, n_dense, seed=0)
    n_nodes = sum(p.n for _, p in parts)
    n_edges = sum(p.m for _, p in parts)
    log(f"batch: {n_nodes} nodes, {n_edges} edges in {len(parts)} contexts; uploading")
    # distinct generator keys: the contexts' node and edge ids overlap
    samplers = [Sampler(p, C, seed=seed + k, burn_in=0) for k, (_, p) in enumerate(parts)]
    alg = sum(dual_bytes(p, C) for _, p in parts)
    pbytes = sum(primal_bytes(p, C) for _, p in parts)
    sizes = [(q, p.n, p.m) for q, p in parts]
    del parts
    for s in samplers:
        s.init()
    tuning = []
    for (q, _, _), s in zip(sizes, samplers):
        t = pdg.pdg_tune(s.ctx, 5).as_dict()
        t["q"] = q
        tuning.append(t)
    log(f"tuned: {tuning}")
    group = SamplerGroup(samplers)
    for _ in range(warmup):
        group.dual_phase()
        group.primal_phase()
    stream = torch.cuda.current_stream()
    # per-phase times from eager launches (HIP events around each phase)
    _, dual_ms, primal_ms, _ = timed_sweeps(group, 10, stream)
    graph = pdg.pdg_graph_create([s.ctx for s in samplers], K)
    pdg.pdg_graph_launch(graph)  # warm
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps // K):
        pdg.pdg_graph_launch(graph)
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = a.elapsed_time(b)
    pdg.pdg_graph_destroy(graph)
    dense = dense_gather_experiment(samplers[0], n_dense * 2048, 2048, C, stream)
    for s in samplers:
        s.sync()
        s.close()
    updates = C * (n_nodes + n_edges)
    achieved = alg / (dual_ms / 1e3) / 1e9
    p_gbs = pbytes / (primal_ms / 1e3) / 1e9
    out = {
        "metric": "chain*(|V|+|E|) updates/s", "value": updates * steps / (total_ms / 1e3),
        "unit": "updates/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": total_ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE, "data": "synthetic",
        "config": {"workload": f"batched uneven: {n_graphs} graphs ({n_dense} dense binary "
                               f"N=2048), q in {{2,3,5}}, FP32 tables, {C} chains",
                   "layout": f"one context per state count ({len(samplers)}), sweeps replayed "
                             f"from one HIP graph of {K} sweeps of every context",
                   "contexts": [{"q": q, "nodes": n, "edges": m} for q, n, m in sizes],
                   "nodes": n_nodes, "edges": n_edges, "chains": C, "seed": seed,
                   "tuning": tuning, "dual_ms_eager": dual_ms, "primal_ms_eager": primal_ms,
                   "dense_gather": dense,
                   "wall_s": wall, "kernel_sources": kernel_digest()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profile_traffic("batched_uneven_sweep_kernels.txt", "dual_phase"),
                     "algorithmic_bytes": alg, "kernel": "dual phase (one launch per state count)"},
        "roofline_primal": {"bound": "hbm", "achieved": p_gbs, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": p_gbs / HBM_PEAK_GBS,
                            "traffic": profile_traffic("batched_uneven_sweep_kernels.txt",
                                                       "primal_phase"),
                            "kernel": "primal phase (per state count, with hub kernels)",
                            "algorithmic_bytes": pbytes},
    }
    if not args.no_cpu_baseline:
        small = W.batched_uneven(16, 1, seed=0)
        out["cpu_baseline"] = cpu_baseline(
            small, C, seed, f"20 sweeps of a 16-graph batch of the same recipe ({small.m} edges)",
            sweeps=20)
    return out


MLP_FLOP_PER_ROW = 2 * (96 * 256 + 256 * 256 + 256 * 64)
BF16_PEAK = 2.5e15


def run_learned(args):
    """Learned block proposal on the 512 x 512 grid (128 chains): ESS/s of
    learned step + plain sweep against plain sweeps, at equal marginal error."""
    import torch
    from paper_1611_06684_amd import learned as L
    from paper_1611_06684_amd import pdg_block as pb
    from paper_1611_06684_amd.pdg import Sampler
    iters = 2000 if args.steps is None else args.steps
    warmup = 500 if args.warmup is None else args.warmup
    side, C, seed = 512, 128, 0
    model = L.grid_model(side, seed=0)
    log("reference marginals (independent plain chains)")
    p_ref = L.reference_marginals(model, C, 100, 500, 4000)
    s = Sampler(model, C, seed=seed, burn_in=0)
    s.init()
    s.sweep(warmup)
    bp = pb.BlockProposal(s, model, side, side, init_seed=0)
    log("collecting training rows")
    X, T = L.collect_training_rows(s, bp, snapshots=2, gap=50)
    n_rows = X.shape[0]
    losses, train_s = L.train(bp, X, T, epochs=args.epochs, log=log)
    del X, T
    # the network alone: one forward over every block and chain
    st = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        pb.pdg_mlp_forward(bp.wbf.data_ptr(), bp.w32.data_ptr(), bp.rows, bp.x_in.data_ptr(),
                           bp.logits.data_ptr(), stream=bp.stream)
    a.record(st)
    for _ in range(20):
        pb.pdg_mlp_forward(bp.wbf.data_ptr(), bp.w32.data_ptr(), bp.rows, bp.x_in.data_ptr(),
                           bp.logits.data_ptr(), stream=bp.stream)
    b.record(st)
    b.synchronize()
    mlp_ms = a.elapsed_time(b) / 20
    ms_plain = L.time_iterations(s, None, 200)
    ms_learned = L.time_iterations(s, bp, 200)
    rng = np.random.default_rng(1)
    nodes = np.sort(rng.choice(model.n, size=256, replace=False))
    log("ESS runs")
    ess_p, mp = L.ess_run(s, None, iters, nodes)
    _, _, acc0, prop0 = pb.pdg_blk_info(bp.blk, s.ctx)
    ess_l, ml = L.ess_run(s, bp, iters, nodes)
    _, _, acc1, prop1 = pb.pdg_blk_info(bp.blk, s.ctx)
    bp.close()
    s.close()
    med_p, med_l = float(np.median(ess_p)), float(np.median(ess_l))
    esss_p = med_p / (iters * ms_plain / 1e3)
    esss_l = med_l / (iters * ms_learned / 1e3)
    err_p = float(np.abs(mp - p_ref).mean())
    err_l = float(np.abs(ml - p_ref).mean())
    flops = bp.rows * MLP_FLOP_PER_ROW
    achieved = flops / (mlp_ms / 1e3)
    return {
        "metric": "ESS/s of the learned block proposal (median over nodes) at marginal error <= 0.01",
        "value": esss_l, "unit": "effective samples/s",
        "n_gpus": 1, "steps": iters, "warmup": warmup,
        "ms_per_step": ms_learned, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 network, f64 MH", "data": "synthetic",
        "config": {"workload": f"learned proposal: {side}x{side} binary grid, J~U(0,0.35), "
                               f"h~N(0,0.3), 8x8 blocks, {C} chains",
                   "plain_ess_per_s": esss_p, "ratio_learned_over_plain": esss_l / esss_p,
                   "ess_median": {"plain": med_p, "learned": med_l},
                   "ess_p10": {"plain": float(np.percentile(ess_p, 10)),
                               "learned": float(np.percentile(ess_l, 10))},
                   "ms_per_iteration": {"plain": ms_plain, "learned": ms_learned},
                   "marginal_error": {"plain": err_p, "learned": err_l},
                   "acceptance": (acc1 - acc0) / max(prop1 - prop0, 1),
                   "training": {"rows": n_rows, "epochs": args.epochs, "loss_per_epoch": losses,
                                "wall_s": train_s},
                   "tracked_nodes": len(nodes)},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK, "unit": "FLOP/s",
                     "frac": achieved / BF16_PEAK, "traffic": None,
                     "kernel": "k_mlp_fwd (proposal network, BF16 MFMA)",
                     "units_per_launch": flops, "launch_ms": mlp_ms},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sampler's "
              "chains would shard across GPUs with no per-sweep communication, but no "
              "multi-GPU path is implemented.", file=sys.stderr)
        sys.exit(2)
    run = {"plain-grid": run_plain, "dynamic-sparse": run_dynamic, "tiny": run_tiny,
           "batched": run_batched, "learned": run_learned}
    out = run[args.workload](args)
    print(json.dumps(out), flush=True)
    if args.copy_mib > 0:
        import torch
        a = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_mib} MiB three times")


if __name__ == "__main__":
    main()
