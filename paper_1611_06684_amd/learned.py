"""The learned-block-proposal workload: train the proposal network on block
states of the plain sampler, then compare effective samples per second of
(learned step + plain sweep) against plain sweeps alone at equal marginal
accuracy (blocking of Sec. 5.4; mixing judged as in Sec. 6).

Workload: 512 x 512 binary grid, phi_e = exp(J_e s s'), J_e ~ U(0, 0.35),
u_i = exp(h_i s), h_i ~ N(0, 0.3), FP32 tables, 8 x 8 blocks (4096), 128
chains.  Everything runs through the C ABI (pdg.h, pdg_block.h); torch holds
buffers, and gathers the tracked nodes' states each iteration for the ESS
(bookkeeping outside the timed iterations).
"""
from __future__ import annotations

import time

import numpy as np

from . import diagnostics as dg
from . import workloads as W


def grid_model(side: int = 512, seed: int = 0) -> W.Model:
    """Draw order: J_e ~ U(0, 0.35) for every edge (grid order), h_i ~ N(0, 0.3)."""
    rng = np.random.default_rng(seed)
    src, dst = W.grid_edges(side, side)
    J = rng.uniform(0.0, 0.35, size=src.shape[0])
    h = rng.normal(0.0, 0.3, size=side * side)
    return W.ising_model(src, dst, J, h, side * side, "f32", name=f"learned_grid_{side}")


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def reference_marginals(model, C, seed, burn, sweeps):
    """p(x_i = 1) from plain sweeps (counters after burn-in)."""
    from .pdg import Sampler
    s = Sampler(model, C, seed=seed, burn_in=burn)
    s.init()
    s.sweep(burn + sweeps)
    p, n = s.marginals()
    out = p.cpu().numpy()[:, 1]
    s.close()
    return out


def collect_training_rows(sampler, bp, snapshots, gap):
    """Rows (inputs, targets) from `snapshots` states of the plain chain, `gap`
    sweeps apart: nb * C rows per snapshot."""
    import torch
    X = torch.empty((snapshots * bp.rows, 96), dtype=torch.int16, device=sampler.dev)
    T = torch.empty((snapshots * bp.rows, 64), dtype=torch.uint8, device=sampler.dev)
    for k in range(snapshots):
        sampler.sweep(gap)
        bp.sample_training_rows(X[k * bp.rows:(k + 1) * bp.rows], T[k * bp.rows:(k + 1) * bp.rows])
    return X, T


def train(bp, X, T, epochs=2, batch=8192, lr=1e-3, seed=0, log=None):
    """Adam on shuffled minibatches; returns the loss of the last batch of each
    epoch and the wall time."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    R = X.shape[0]
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(R, generator=g).to(X.device)
        for k in range(0, R - batch + 1, batch):
            idx = perm[k:k + batch]
            bp.train_step(X[idx].contiguous(), T[idx].contiguous(), lr=lr)
        losses.append(float(bp.loss.cpu()[0]))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4f}")
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def time_iterations(sampler, bp, iters):
    """Milliseconds per iteration: a plain sweep, preceded by a learned step when
    bp is given (HIP events on the sampler's stream)."""
    import torch
    a, b = _events()
    st = torch.cuda.current_stream()
    a.record(st)
    for _ in range(iters):
        if bp is not None:
            bp.step()
        sampler.sweep(1)
    b.record(st)
    b.synchronize()
    return a.elapsed_time(b) / iters


def ess_run(sampler, bp, iters, nodes):
    """Indicator series of the tracked nodes over `iters` iterations: returns
    (ESS per node, marginals from the counters over the run)."""
    import torch
    sampler.reset_marginals()
    idx = torch.as_tensor(nodes, device=sampler.dev)
    trace = torch.empty((iters, len(nodes), sampler.C), dtype=torch.uint8, device=sampler.dev)
    for t in range(iters):
        if bp is not None:
            bp.step()
        sampler.sweep(1)
        trace[t] = sampler.state().index_select(0, idx)
    p, _ = sampler.marginals()
    tr = trace.cpu().numpy()
    ess = np.array([dg.ess(tr[:, k, :].T.astype(np.float64)) for k in range(len(nodes))])
    return ess, p.cpu().numpy()[:, 1]
