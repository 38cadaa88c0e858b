"""Sweeps replayed from a captured HIP graph (``-m gpu``): the graph's tick
kernel advances a device-resident sweep counter that the phase kernels read,
so every replay draws new numbers; states, counters and sweep counters must
equal eager phase launches bit for bit after every replay, with eager work and
synchronisations between the replays; edits invalidate a graph."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1611_06684_amd import workloads as W
from tests.test_gpu_parity import _hub_graph

pytestmark = pytest.mark.gpu


def _eager(s, k):
    for _ in range(k):
        s.dual_phase()
        s.primal_phase()


def _same(a, b):
    assert a.t == b.t
    assert np.array_equal(a.state().cpu().numpy(), b.state().cpu().numpy())
    ca, na = a.counts()
    cb, nb = b.counts()
    assert na == nb and np.array_equal(ca, cb)


@pytest.mark.parametrize("case", ["mixed_C20", "batch_by_states_C8", "hubs_C100", "small_C5"])
def test_graph_replays_equal_eager_sweeps(case):
    from paper_1611_06684_amd import pdg
    from paper_1611_06684_amd.pdg import Sampler
    if case == "mixed_C20":
        models, C = [W.random_graph(400, 1200, [2, 4, 7], seed=1, dtype="f32")], 20
    elif case == "batch_by_states_C8":
        batch = W.batched_uneven(30, 2, seed=1, n_min=20, n_max=300, dense_n=300)
        models, C = [m for _, m in W.group_by_states(batch)], 8
    elif case == "hubs_C100":
        models, C = [_hub_graph(600, [2], 2, 10)], 100
    else:  # small enough for the one-launch form in pdg_sweep
        models, C = [W.random_graph(30, 50, [2, 3], seed=4, dtype="f32")], 5
    K = 6
    graphed = [Sampler(m, C, seed=3 + k, burn_in=4) for k, m in enumerate(models)]
    eager = [Sampler(m, C, seed=3 + k, burn_in=4) for k, m in enumerate(models)]
    for s in graphed + eager:
        s.init()
    g = pdg.pdg_graph_create([s.ctx for s in graphed], K)
    try:
        for rep in range(4):
            pdg.pdg_graph_launch(g)
            for s in eager:
                _eager(s, K)
            for a, b in zip(graphed, eager):
                _same(a, b)
            # eager work between the replays, on both sides
            for s in graphed + eager:
                s.sweep(2)
                s.sync()
        # an edit invalidates the captured graph
        s0 = graphed[0]
        s0.remove_edges(s0.uids[:1])
        with pytest.raises(pdg.PdgError) as e:
            pdg.pdg_graph_launch(g)
        assert e.value.code == pdg.PDG_ESTATE
    finally:
        pdg.pdg_graph_destroy(g)
    for s in graphed + eager:
        s.close()
