"""Mixing of the primal-dual sampler by the potential scale reduction factor
(Sec. 6): a 50 x 50 Ising grid with uniform coupling beta and no field, 10
chains from random states; the PSRF of every node's indicator [x_i = 1] is
taken over the second half of the first T sweeps, the largest over nodes is the
grid's PSRF at T, and the mixing time is the first T after which it stays below
1.01.

    python -m paper_1611_06684_amd.mixing [--betas 0.1,0.2,...] [--max-sweeps N]

Prints one JSON line per beta.  The sweeps run on the GPU through the C ABI;
the chains' running sums of x are kept on the device (a torch add per sweep:
bookkeeping, not sampler arithmetic) and copied out at the evaluation points.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import diagnostics as dg
from . import workloads as W


def uniform_ising(side: int, beta: float, dtype: str = "f64") -> W.Model:
    """side x side open grid, phi_e = exp(beta s s'), no unary field."""
    src, dst = W.grid_edges(side, side)
    return W.ising_model(src, dst, np.full(src.shape[0], beta), np.zeros(side * side),
                         side * side, dtype, name=f"ising_{side}x{side}_beta{beta}")


def eval_points(max_sweeps: int, first: int = 8, ratio: float = 1.05):
    pts, t = [], float(first)
    while int(t) <= max_sweeps:
        if not pts or int(t) != pts[-1]:
            pts.append(int(t))
        t *= ratio
    if pts[-1] != max_sweeps:
        pts.append(max_sweeps)
    return pts


def psrf_trace(beta: float, side: int = 50, chains: int = 10, seed: int = 0,
               max_sweeps: int = 20000, threshold: float = 1.01):
    """PSRF over the second half of the first T sweeps at geometric T (5 %
    apart) up to max_sweeps; returns (times, psrf, mixing time or None)."""
    import torch
    from .pdg import Sampler
    model = uniform_ising(side, beta)
    s = Sampler(model, chains, seed=seed)
    s.init()
    pts = eval_points(max_sweeps)
    need = sorted(set(pts) | {p // 2 for p in pts})
    cum = torch.zeros((model.n, chains), dtype=torch.int32, device=s.dev)
    snaps = {0: np.zeros((model.n, chains), np.int64)}
    t = 0
    for target in need:
        while t < target:
            s.sweep(1)
            cum += s.state()
            t += 1
        snaps[target] = cum.cpu().numpy().astype(np.int64)
    s.close()
    vals = []
    for T in pts:
        h = T // 2
        L = T - h
        means = ((snaps[T] - snaps[h]) / L).T  # [chains, nodes]
        vals.append(float(dg.psrf_binary(means, L).max()))
    return pts, vals, dg.mixing_time(pts, vals, threshold)


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--betas", default="0.1,0.15,0.2,0.25,0.3,0.35,0.4,0.45,0.5")
    p.add_argument("--max-sweeps", type=int, default=20000)
    p.add_argument("--side", type=int, default=50)
    p.add_argument("--chains", type=int, default=10)
    p.add_argument("--seed", type=int, default=0)
    a = p.parse_args(argv)
    for beta in (float(b) for b in a.betas.split(",")):
        t0 = time.perf_counter()
        pts, vals, mt = psrf_trace(beta, a.side, a.chains, a.seed, a.max_sweeps)
        print(json.dumps({"beta": beta, "side": a.side, "chains": a.chains,
                          "max_sweeps": a.max_sweeps, "mixing_time_sweeps": mt,
                          "final_psrf": vals[-1], "wall_s": time.perf_counter() - t0,
                          "trace": [[T, round(v, 5)] for T, v in zip(pts, vals)][::8]}),
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
