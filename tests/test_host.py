"""CPU checks of host-side logic: the workload generators' structure and the
benchmark's one-GPU contract."""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np

from paper_1611_06684_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_batched_uneven_is_a_disjoint_union():
    m = W.batched_uneven(12, 2, seed=3, n_min=20, n_max=200, dense_n=30)
    no, eo = m.meta["node_off"], m.meta["edge_off"]
    assert no[0] == 0 and no[-1] == m.n and eo[0] == 0 and eo[-1] == m.m
    for g in range(12):
        a, b = no[g], no[g + 1]
        src, dst = m.src[eo[g]:eo[g + 1]], m.dst[eo[g]:eo[g + 1]]
        # every edge stays inside its graph, no self-loops, one q per graph
        assert ((src >= a) & (src < b) & (dst >= a) & (dst < b)).all()
        assert (src != dst).all()
        assert len(set(m.q[a:b].tolist())) == 1
        qg = int(m.q[a])
        L = m.Lam[eo[g]:eo[g + 1]]
        assert not L[:, qg:, :].any() and not L[:, :, qg:].any()
        if g < 2:  # dense binary graphs: complete, Ising tables
            n = b - a
            assert qg == 2 and len(src) == n * (n - 1) // 2
            assert np.allclose(L[:, 0, 0], L[:, 1, 1]) and np.allclose(L[:, 0, 1], -L[:, 0, 0])
        else:
            assert qg in (2, 3, 5)
    # unaries are zero past each node's states
    beyond = np.arange(m.q_max)[None, :] >= m.q[:, None]
    assert not m.lam[beyond].any()


def test_batched_uneven_is_seeded():
    a = W.batched_uneven(6, 1, seed=5, n_min=20, n_max=100, dense_n=12)
    b = W.batched_uneven(6, 1, seed=5, n_min=20, n_max=100, dense_n=12)
    for f in ("q", "lam", "src", "dst", "Lam"):
        assert np.array_equal(getattr(a, f), getattr(b, f))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _log_density(model, x):
    """Unnormalised log-density of one state: unaries plus pairwise log-tables."""
    e = np.arange(model.m)
    return (model.lam[np.arange(model.n), x].astype(np.float64).sum()
            + model.Lam[e, x[model.src], x[model.dst]].astype(np.float64).sum())


def test_group_by_states_partitions_the_batch():
    m = W.batched_uneven(14, 2, seed=7, n_min=20, n_max=150, dense_n=24)
    groups = W.group_by_states(m)
    assert [q for q, _ in groups] == sorted({int(v) for v in m.q})
    nodes = np.concatenate([g.meta["node_map"] for _, g in groups])
    edges = np.concatenate([g.meta["edge_map"] for _, g in groups])
    assert np.array_equal(np.sort(nodes), np.arange(m.n))
    assert np.array_equal(np.sort(edges), np.arange(m.m))
    for q, g in groups:
        nm, em = g.meta["node_map"], g.meta["edge_map"]
        assert g.q_max == q and (g.q == q).all()
        assert np.array_equal(nm[g.src], m.src[em]) and np.array_equal(nm[g.dst], m.dst[em])
        assert np.array_equal(g.lam, m.lam[nm, :q])
        assert np.array_equal(g.Lam, m.Lam[em, :q, :q])
    # the batch's log-density is the sum of the groups' at every state
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = (rng.random(m.n) * m.q).astype(np.int64)
        parts = sum(_log_density(g, x[g.meta["node_map"]]) for _, g in groups)
        assert abs(_log_density(m, x) - parts) <= 1e-9 * (1 + abs(parts))


def test_dual_bytes_counts_each_edge_by_its_states():
    """The batched roofline's algorithmic bytes: per edge 32 B of metadata and
    sign word, 8 D of thresholds, 2 C of endpoint states and 8 D of mask words
    written, with D = (q_src - 1)(q_dst - 1)."""
    sys.path.insert(0, ROOT)
    import bench
    q = np.array([2, 3, 5, 5], np.int32)
    src = np.array([0, 1, 2, 0], np.int32)
    dst = np.array([1, 2, 3, 3], np.int32)
    m = W.Model(q, np.zeros((4, 5), np.float32), src, dst, np.zeros((4, 5, 5), np.float32))
    C = 8
    Ds = [1 * 2, 2 * 4, 4 * 4, 1 * 4]
    assert bench.dual_bytes(m, C) == sum(32 + 2 * C + 16 * d for d in Ds)


def test_byte_models_of_chain_major_words():
    """With 17..32 chains and q_max >= 6 each record carries one 64-bit word per
    chain: 8 C bytes per record written by the dual (two records per edge) and
    read by the primal, in place of 4 D bytes of 32-bit mask words (8 D per
    block of 64 chains above 32 chains)."""
    sys.path.insert(0, ROOT)
    import bench
    q = np.array([6, 6, 2], np.int32)
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 2], np.int32)
    m = W.Model(q, np.zeros((3, 6), np.float32), src, dst, np.zeros((2, 6, 6), np.float32))
    Ds = [5 * 5, 5 * 1]
    for C, chain_major in [(16, False), (17, True), (32, True), (33, False), (130, False)]:
        if chain_major:
            words = [8 * C] * 2
        elif C <= 32:
            words = [4 * d for d in Ds]
        else:  # one 64-bit mask per entry and block of 64 chains
            words = [8 * d * ((C + 63) // 64) for d in Ds]
        assert bench.chain_major(m, C) == chain_major
        assert bench.dual_bytes(m, C) == sum(32 + 2 * C + 8 * d + 2 * w for d, w in zip(Ds, words))
        assert bench.primal_bytes(m, C) == (2 * sum(8 * d + w for d, w in zip(Ds, words))
                                            + 3 * (16 * 6 + C + 8))


def test_batch_by_states_equals_grouped_batch():
    """The per-state-count batch generator draws the same graphs, tables and
    unaries as the padded one-model batch split by state count."""
    from paper_1611_06684_amd import workloads as W
    for args in [(30, 2, 1, 20, 300, 40), (12, 1, 5, 100, 2000, 64)]:
        a = W.group_by_states(W.batched_uneven(*args[:3], n_min=args[3], n_max=args[4],
                                               dense_n=args[5]))
        b = W.batched_by_states(*args[:3], n_min=args[3], n_max=args[4], dense_n=args[5])
        assert [q for q, _ in a] == [q for q, _ in b]
        for (q, x), (_, y) in zip(a, b):
            for f in ("q", "lam", "src", "dst", "Lam"):
                assert np.array_equal(getattr(x, f), getattr(y, f)), (q, f)
            assert np.array_equal(x.meta["graphs"], y.meta["graphs"])
