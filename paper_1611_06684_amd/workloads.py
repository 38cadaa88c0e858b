"""Seeded synthetic inputs: graphs, log-factor tables, unaries and churn batches.

This module holds no arithmetic of the sampler.  It is the only code that both
the GPU path (bench, tests) and the CPU oracle (tests) consume.  Every generator
draws from ``numpy.random.default_rng(seed)`` in a fixed order, stated in each
docstring, so the same seed gives the same model everywhere.

Conventions (the paper's experiments, Sec. 6, define the workload families):
  * node states x in {0..q-1}; Ising spins s = 2x - 1;
  * ``Lam[e][a][b]`` = log phi_e(x_src = a, x_dst = b), row = src state;
  * ``lam[i][a]`` = log u_i(a);
  * entries beyond a node's q are zero and never read;
  * N(mu, s) means standard deviation s.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Model:
    q: np.ndarray          # int32 [n]
    lam: np.ndarray        # [n][q_max], dtype = table precision
    src: np.ndarray        # int32 [m]
    dst: np.ndarray        # int32 [m]
    Lam: np.ndarray        # [m][q_max][q_max], dtype = table precision
    name: str = "model"
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q.shape[0])

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    @property
    def q_max(self) -> int:
        return int(self.lam.shape[1])

    @property
    def fp64(self) -> bool:
        return self.Lam.dtype == np.float64

    def subset_edges(self, idx) -> "Model":
        idx = np.asarray(idx)
        return Model(self.q, self.lam, self.src[idx], self.dst[idx], self.Lam[idx],
                     self.name, dict(self.meta))


def _np_dtype(dtype: str):
    return {"f32": np.float32, "f64": np.float64}[dtype]


def grid_edges(H: int, W: int):
    """Open-boundary 4-neighbour grid, node = r*W + c.  All horizontal edges in
    row-major order, then all vertical ones; src is the left/top endpoint."""
    r, c = np.meshgrid(np.arange(H), np.arange(W - 1), indexing="ij")
    hs = (r * W + c).ravel()
    hd = hs + 1
    r, c = np.meshgrid(np.arange(H - 1), np.arange(W), indexing="ij")
    vs = (r * W + c).ravel()
    vd = vs + W
    return (np.concatenate([hs, vs]).astype(np.int32),
            np.concatenate([hd, vd]).astype(np.int32))


def ising_grid(H: int, W: int, seed: int = 0, J_half_range: float = 0.3,
               h_std: float = 0.5, dtype: str = "f64") -> Model:
    """Binary grid with phi_e = exp(J_e s_i s_j), u_i = exp(h_i s_i).
    Draw order: J_e ~ U(-J_half_range, J_half_range) for every edge, then
    h_i ~ N(0, h_std) for every node."""
    rng = np.random.default_rng(seed)
    src, dst = grid_edges(H, W)
    J = rng.uniform(-J_half_range, J_half_range, size=src.shape[0])
    h = rng.normal(0.0, h_std, size=H * W)
    return ising_model(src, dst, J, h, H * W, dtype, name=f"ising_grid_{H}x{W}")


def ising_model(src, dst, J, h, n, dtype="f64", name="ising") -> Model:
    s = np.array([-1.0, 1.0])
    Lam = J[:, None, None] * s[None, :, None] * s[None, None, :]
    lam = h[:, None] * s[None, :]
    dt = _np_dtype(dtype)
    return Model(np.full(n, 2, np.int32), lam.astype(dt), np.asarray(src, np.int32),
                 np.asarray(dst, np.int32), Lam.astype(dt), name)


def table_grid(H: int, W: int, q: int, seed: int = 0, pair_std: float = 0.2,
               unary_std: float = 1.0, dtype: str = "f32") -> Model:
    """q-state grid with iid Gaussian log-tables.  Draw order: Lam [m][q][q]
    ~ N(0, pair_std), then lam [n][q] ~ N(0, unary_std); generated in the table
    precision."""
    rng = np.random.default_rng(seed)
    src, dst = grid_edges(H, W)
    dt = _np_dtype(dtype)
    Lam = (rng.standard_normal((src.shape[0], q, q), dtype=dt) * dt(pair_std)).astype(dt)
    lam = (rng.standard_normal((H * W, q), dtype=dt) * dt(unary_std)).astype(dt)
    return Model(np.full(H * W, q, np.int32), lam, src, dst, Lam, f"grid_{H}x{W}_q{q}")


def chung_lu_weights(n: int, gamma: float = 2.5, mean_deg: float = 8.0) -> np.ndarray:
    """Expected degrees w_i proportional to (i + i0)^(-1/(gamma-1)), scaled to
    mean ``mean_deg``, with i0 chosen so that w_0 = sqrt(sum w)."""
    alpha = 1.0 / (gamma - 1.0)
    i = np.arange(n, dtype=np.float64)
    target = np.sqrt(n * mean_deg)

    def w0(i0):
        base = (i + i0) ** (-alpha)
        return n * mean_deg * base[0] / base.sum()

    lo, hi = 1e-6, float(n)
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if w0(mid) > target:
            lo = mid
        else:
            hi = mid
    i0 = np.sqrt(lo * hi)
    base = (i + i0) ** (-alpha)
    return n * mean_deg * base / base.sum()


def chung_lu(n: int, q: int, seed: int = 0, gamma: float = 2.5, mean_deg: float = 8.0,
             pair_std: float = 0.15, unary_std: float = 1.0, dtype: str = "f32") -> Model:
    """Chung-Lu power-law graph.  Draw order: M = round(n mean_deg / 2) src
    endpoints iid proportional to w, then M dst endpoints; self-loops and repeated
    unordered pairs are dropped (first occurrence kept, draw order preserved);
    then Lam [m][q][q] ~ N(0, pair_std), then lam [n][q] ~ N(0, unary_std)."""
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, gamma, mean_deg)
    p = w / w.sum()
    M = int(round(n * mean_deg / 2))
    s = rng.choice(n, size=M, p=p)
    d = rng.choice(n, size=M, p=p)
    keep = s != d
    s, d = s[keep], d[keep]
    key = np.minimum(s, d).astype(np.int64) * n + np.maximum(s, d)
    _, first = np.unique(key, return_index=True)
    first.sort()
    src, dst = s[first].astype(np.int32), d[first].astype(np.int32)
    dt = _np_dtype(dtype)
    Lam = (rng.standard_normal((src.shape[0], q, q), dtype=dt) * dt(pair_std)).astype(dt)
    lam = (rng.standard_normal((n, q), dtype=dt) * dt(unary_std)).astype(dt)
    return Model(np.full(n, q, np.int32), lam, src, dst, Lam, f"chung_lu_{n}_q{q}",
                 {"weights": w})


def random_graph(n: int, m: int, qs, seed: int = 0, pair_std: float = 0.5,
                 unary_std: float = 1.0, dtype: str = "f64", allow_parallel=True) -> Model:
    """Small mixed-q test graph.  Draw order: q_i uniform from ``qs`` for every
    node, then m (src, dst) pairs uniform without self-loops (dst redrawn as
    (src + 1 + U{0..n-2}) mod n), then Lam, then lam, all N(0, std)."""
    rng = np.random.default_rng(seed)
    q = rng.choice(np.asarray(qs), size=n).astype(np.int32)
    qm = int(max(qs))
    src = rng.integers(0, n, size=m)
    dst = (src + 1 + rng.integers(0, n - 1, size=m)) % n
    dt = _np_dtype(dtype)
    Lam = rng.normal(0.0, pair_std, size=(m, qm, qm))
    lam = rng.normal(0.0, unary_std, size=(n, qm))
    for e in range(m):
        Lam[e, q[src[e]]:, :] = 0.0
        Lam[e, :, q[dst[e]]:] = 0.0
    for i in range(n):
        lam[i, q[i]:] = 0.0
    return Model(q, lam.astype(dt), src.astype(np.int32), dst.astype(np.int32),
                 Lam.astype(dt), f"random_{n}_{m}")



def batched_uneven(n_graphs: int, n_dense: int, seed: int = 0, n_min: int = 100,
                   n_max: int = 50000, dense_n: int = 2048, dtype: str = "f32") -> Model:
    """A batch of independent graphs as one model (disjoint union; node ids of
    graph g start at meta["node_off"][g], its edges at meta["edge_off"][g]).
    Sparse graphs: N ~ logU[n_min, n_max], mean degree d ~ U{3..12}, q ~ U{2,3,5}
    per graph, N d / 2 endpoint pairs uniform within the graph (a self-loop's
    dst moves to the next node), Lam ~ N(0, 0.2); dense graphs (the first
    n_dense): complete binary graphs on dense_n nodes with Ising tables
    J ~ N(0, 0.5 / sqrt(dense_n)); lam ~ N(0, 1) everywhere.  Draw order: per
    graph in order, its size and q (sparse) then its edges, tables, unaries."""
    rng = np.random.default_rng(seed)
    dt = _np_dtype(dtype)
    qm = 5
    qs, lams, srcs, dsts, Lams = [], [], [], [], []
    node_off, edge_off = [0], [0]
    for g in range(n_graphs):
        base = node_off[-1]
        if g < n_dense:
            N = dense_n
            q = np.full(N, 2, np.int32)
            iu, ju = np.triu_indices(N, 1)
            J = rng.normal(0.0, 0.5 / np.sqrt(N), size=iu.shape[0])
            s = np.array([-1.0, 1.0])
            L = np.zeros((iu.shape[0], qm, qm))
            L[:, :2, :2] = J[:, None, None] * s[None, :, None] * s[None, None, :]
            src, dst = iu, ju
        else:
            N = int(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
            d = int(rng.integers(3, 13))
            qg = int(rng.choice([2, 3, 5]))
            q = np.full(N, qg, np.int32)
            M = N * d // 2
            src = rng.integers(0, N, size=M)
            dst = rng.integers(0, N, size=M)
            dst = np.where(src == dst, (dst + 1) % N, dst)
            L = np.zeros((M, qm, qm))
            L[:, :qg, :qg] = rng.normal(0.0, 0.2, size=(M, qg, qg))
        lam = np.zeros((N, qm))
        lam[:, :int(q[0])] = rng.normal(0.0, 1.0, size=(N, int(q[0])))
        qs.append(q)
        lams.append(lam)
        srcs.append((src + base).astype(np.int32))
        dsts.append((dst + base).astype(np.int32))
        Lams.append(L.astype(dt))
        node_off.append(base + N)
        edge_off.append(edge_off[-1] + len(src))
    return Model(np.concatenate(qs), np.concatenate(lams).astype(dt), np.concatenate(srcs),
                 np.concatenate(dsts), np.concatenate(Lams), f"batch_{n_graphs}",
                 {"node_off": np.array(node_off), "edge_off": np.array(edge_off)})

def batched_by_states(n_graphs: int, n_dense: int, seed: int = 0, n_min: int = 100,
                      n_max: int = 50000, dense_n: int = 2048, dtype: str = "f32") -> list:
    """The batch of ``batched_uneven`` (same recipe, same draws in the same
    order) built directly as one model per state count, tables q x q, so no
    table is padded to the largest q.  Returns [(q, model)] in increasing q with
    ``meta["graphs"]`` the batch indices of each model's graphs; equal to
    ``group_by_states(batched_uneven(...))`` for the same arguments."""
    rng = np.random.default_rng(seed)
    dt = _np_dtype(dtype)
    parts = {}
    for g in range(n_graphs):
        if g < n_dense:
            N, q = dense_n, 2
            iu, ju = np.triu_indices(N, 1)
            J = rng.normal(0.0, 0.5 / np.sqrt(N), size=iu.shape[0])
            s = np.array([-1.0, 1.0], dtype=dt)
            L = J.astype(dt)[:, None, None] * s[None, :, None] * s[None, None, :]
            src, dst = iu, ju
        else:
            N = int(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
            d = int(rng.integers(3, 13))
            q = int(rng.choice([2, 3, 5]))
            M = N * d // 2
            src = rng.integers(0, N, size=M)
            dst = rng.integers(0, N, size=M)
            dst = np.where(src == dst, (dst + 1) % N, dst)
            L = rng.normal(0.0, 0.2, size=(M, q, q)).astype(dt)
        lam = rng.normal(0.0, 1.0, size=(N, q)).astype(dt)
        p = parts.setdefault(q, {"n": 0, "src": [], "dst": [], "Lam": [], "lam": [], "graphs": []})
        p["src"].append((src + p["n"]).astype(np.int32))
        p["dst"].append((dst + p["n"]).astype(np.int32))
        p["Lam"].append(L)
        p["lam"].append(lam)
        p["graphs"].append(g)
        p["n"] += N
    out = []
    for q in sorted(parts):
        p = parts[q]
        out.append((q, Model(np.full(p["n"], q, np.int32), np.concatenate(p["lam"]),
                             np.concatenate(p["src"]), np.concatenate(p["dst"]),
                             np.concatenate(p["Lam"]), f"batch_{n_graphs}_q{q}",
                             {"graphs": np.array(p["graphs"])})))
        parts[q] = None
    return out


def group_by_states(batch: Model) -> list:
    """Splits a batch of independent graphs (``meta`` with ``node_off`` and
    ``edge_off``, every node of a graph with the same state count) into one
    model per state count q, tables cut to q x q and node ids renumbered
    consecutively in graph order.  Returns [(q, model)] in increasing q; each
    model's ``meta["graphs"]`` lists the batch's graph indices it holds and
    ``meta["node_map"]`` / ``meta["edge_map"]`` the batch's node and edge index of
    each of its nodes and edges.  The graphs do not interact, so sampling the
    groups as separate models samples the batch."""
    no, eo = batch.meta["node_off"], batch.meta["edge_off"]
    gq = batch.q[no[:-1]]
    out = []
    for q in sorted(set(int(v) for v in gq)):
        graphs = np.flatnonzero(gq == q)
        nmap = np.concatenate([np.arange(no[g], no[g + 1]) for g in graphs]).astype(np.int64)
        emap = np.concatenate([np.arange(eo[g], eo[g + 1]) for g in graphs]).astype(np.int64)
        if np.any(batch.q[nmap] != q):
            raise ValueError("a graph of the batch mixes state counts")
        new_id = np.full(batch.n, -1, np.int64)
        new_id[nmap] = np.arange(nmap.shape[0])
        sub = Model(batch.q[nmap].copy(), np.ascontiguousarray(batch.lam[nmap, :q]),
                    new_id[batch.src[emap]].astype(np.int32),
                    new_id[batch.dst[emap]].astype(np.int32),
                    np.ascontiguousarray(batch.Lam[emap, :q, :q]), f"{batch.name}_q{q}",
                    {"graphs": graphs, "node_map": nmap, "edge_map": emap})
        out.append((q, sub))
    return out


class Churn:
    """Edge churn for dynamic graphs: each batch removes ``frac`` of the live
    edges uniformly without replacement and inserts as many new edges whose
    endpoints are drawn iid proportional to ``weights`` (a self-loop's dst is
    moved to the next node), with fresh tables Lam ~ N(0, pair_std).
    Draw order per batch: removal positions, src, dst, tables."""

    def __init__(self, n: int, q: int, weights, seed: int = 1, frac: float = 0.01,
                 pair_std: float = 0.15, dtype: str = "f32"):
        self.rng = np.random.default_rng(seed)
        self.n, self.q, self.frac, self.pair_std = n, q, frac, pair_std
        w = np.asarray(weights, np.float64)
        self.p = w / w.sum()
        self.dt = _np_dtype(dtype)

    def next_batch(self, live_uids: np.ndarray):
        """live_uids: the live edges in a fixed order.  Returns (remove_uids,
        src, dst, Lam) for the batch."""
        k = int(round(self.frac * len(live_uids)))
        pos = np.sort(self.rng.choice(len(live_uids), size=k, replace=False))
        s = self.rng.choice(self.n, size=k, p=self.p)
        d = self.rng.choice(self.n, size=k, p=self.p)
        d = np.where(s == d, (d + 1) % self.n, d)
        Lam = (self.rng.standard_normal((k, self.q, self.q), dtype=self.dt)
               * self.dt(self.pair_std)).astype(self.dt)
        return (np.asarray(live_uids)[pos], s.astype(np.int32), d.astype(np.int32), Lam)
