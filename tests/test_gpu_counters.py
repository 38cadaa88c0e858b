"""Marginal counters (a5) and their readout (a7) against the FP64 oracle, one
test per primal kernel shape (``-m gpu``).

FP64 contexts (FP64 exp in the node draw, FP64 decomposition and fields) follow
the oracle's trajectory exactly, so after free-running sweeps from init the
state and every counter must equal the oracle's.  The sweeps are launched one
phase at a time, so small graphs do not take the one-launch path and each case
reaches the kernel it names: the chain count picks the shape (1..16 chains:
k_primal, or k_primal_st for q_max >= 3 with 8 or 16 chains; 17..32:
k_primal32, or k_primal32z for q_max >= 6; 33 or more: k_primal64, ragged chain blocks above 64), and nodes
with more than 256 incidences go through k_hub_pieces + k_hub_finish (its
counters owned by one wave for one chain block, added atomically for more).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1611_06684_amd import workloads as W
from tests.test_gpu_parity import _hub_graph

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    f64 = np.float64
    yield "primal64_q4_C100", W.table_grid(20, 20, 4, seed=1, dtype="f64"), 100
    yield "primal64_mixed_C64", W.random_graph(300, 700, [2, 3, 6], seed=2), 64
    yield "primal32_q5_C20", W.random_graph(200, 500, [5], seed=3), 20
    yield "primal32z_q8_C20", W.random_graph(200, 500, [8], seed=3), 20
    yield "primal32z_q8_C32", W.random_graph(200, 500, [8], seed=4), 32
    yield "primal32z_mixed_q67_C24", W.random_graph(200, 500, [6, 7], seed=12), 24
    yield "primal_st_q35_C8", W.random_graph(300, 800, [3, 5], seed=5), 8
    yield "primal_st_q5_C16", W.random_graph(300, 800, [5], seed=6), 16
    yield "primal_st_q3_C8", W.random_graph(300, 800, [3], seed=7), 8
    yield "primal_q2_C1", W.ising_grid(20, 20, seed=8, J_half_range=0.6), 1
    yield "primal_q2_C8", W.ising_grid(20, 20, seed=9, J_half_range=0.6), 8
    yield "primal_q2_C16", W.ising_grid(20, 20, seed=10, J_half_range=0.6), 16
    yield "primal_mixed_C5", W.random_graph(300, 700, [2, 4, 7], seed=11), 5
    yield "hubs_mixed_C32", _hub_graph(700, [2, 3, 5], 4, 9, f64), 32
    yield "hubs_z_q8_C32", _hub_graph(500, [8], 2, 13, f64), 32
    yield "hubs_q2_C100", _hub_graph(600, [2], 2, 10, f64), 100
    yield "hubs_q4_C16", _hub_graph(900, [4], 3, 8, f64), 16
    yield "hubs_q2_C1", _hub_graph(600, [2], 2, 10, f64), 1


@pytest.mark.parametrize("name,model,C", list(_cases()), ids=[c[0] for c in _cases()])
def test_free_running_counts_exact(name, model, C):
    from paper_1611_06684_amd.pdg import Sampler
    seed, sweeps, burn = 23, 120, 30
    _say(f"[counters] {name} n={model.n} m={model.m} C={C}")
    assert model.fp64
    s = Sampler(model, C, seed=seed, burn_in=burn)
    s.init()
    for _ in range(sweeps):
        s.dual_phase()
        s.primal_phase()
    x_g = s.state().cpu().numpy()
    cnt_g, samples = s.counts()
    p_g, samples2 = s.marginals()
    p_g = p_g.cpu().numpy()
    uid = s.uids.cpu().numpy().view(np.uint64)
    s.close()
    dec = oracle.decompose(model)
    x_o = oracle.init_state(model, C, seed)
    cnt_o, _, _ = oracle.run(model, dec, uid, seed, x_o, 0, sweeps, burn_in=burn)
    assert samples == samples2 == C * (sweeps - burn)
    assert np.array_equal(x_g, x_o), name
    assert np.array_equal(cnt_g, cnt_o.astype(np.int64)), name
    # a7: the readout is count / samples, one FP64 division per entry
    assert np.array_equal(p_g, cnt_o.astype(np.float64) / samples), name
    q_row = np.arange(model.q_max)[None, :] < model.q[:, None]
    assert (p_g[~q_row] == 0).all()
    np.testing.assert_allclose(p_g.sum(axis=1), 1.0, rtol=0, atol=1e-12)


def test_marginals_readout_edge_cases():
    """Before any counted sweep the readout is all zeros with 0 samples; after a
    reset it is zeros again; pdg_sweep (the one-launch path for a small graph)
    and phase launches give the same readout."""
    from paper_1611_06684_amd.pdg import Sampler
    model = W.random_graph(40, 70, [2, 3, 4], seed=31)
    out = []
    for one_launch in (True, False):
        s = Sampler(model, 6, seed=2, burn_in=5)
        s.init()
        p0, n0 = s.marginals()
        assert n0 == 0 and not p0.cpu().numpy().any()
        if one_launch:
            s.sweep(40)
        else:
            for _ in range(40):
                s.dual_phase()
                s.primal_phase()
        p, n = s.marginals()
        cnt, n2 = s.counts()
        assert n == n2 == 6 * 35
        assert np.array_equal(p.cpu().numpy(), cnt / n)
        out.append(p.cpu().numpy())
        s.reset_marginals()
        p3, n3 = s.marginals()
        assert n3 == 0 and not p3.cpu().numpy().any()
        s.close()
    assert np.array_equal(out[0], out[1])
