"""pdg_log_v_noalloc (static workspace, no allocation) against pdg_log_v on the
same state, through the C ABI (``-m gpu``).  Two contexts in a row, the second
smaller, so the second call runs over the first call's leftovers in the shared
workspace; and a graph too large for the workspace is refused without a launch."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1611_06684_amd import workloads as W

pytestmark = pytest.mark.gpu


def _both(model, C, seed):
    import torch
    from paper_1611_06684_amd import pdg
    from paper_1611_06684_amd.pdg import Sampler
    s = Sampler(model, C, seed=seed)
    s.init()
    s.sweep(3)
    s.dual_phase()
    a = torch.full((C,), float("nan"), dtype=torch.float64, device=s.dev)
    b = torch.full((C,), float("nan"), dtype=torch.float64, device=s.dev)
    pdg.pdg_log_v(s.ctx, a.data_ptr())
    pdg.pdg_log_v_noalloc(s.ctx, b.data_ptr())
    s.primal_phase()
    s.sync()
    out = a.cpu().numpy(), b.cpu().numpy()
    s.close()
    return out


def test_noalloc_log_v_matches_log_v_twice_second_smaller():
    big = W.table_grid(300, 260, 4, seed=3)          # 78 000 nodes, 155 440 edges
    small = W.random_graph(500, 1200, [2, 3, 5], seed=4, dtype="f32")
    for model, C in ((big, 100), (small, 20)):
        a, b = _both(model, C, seed=7)
        print(f"  n={model.n} m={model.m} C={C}: log V {a[:3]} / {b[:3]}", flush=True)
        assert np.isfinite(a).all()
        assert np.array_equal(a, b)


def test_noalloc_log_v_refuses_a_graph_beyond_its_workspace():
    import torch
    from paper_1611_06684_amd import pdg
    from paper_1611_06684_amd.pdg import Sampler
    # 2^21 nodes with 100 chains (two chain blocks): 131 072 node rows of
    # 1 KiB alone exceed 64 MiB
    n = 1 << 21
    model = W.Model(np.full(n, 2, np.int32), np.zeros((n, 2), np.float32),
                    np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 2, 2), np.float32))
    s = Sampler(model, 100, seed=1)
    s.init()
    s.dual_phase()
    out = torch.zeros(100, dtype=torch.float64, device=s.dev)
    with pytest.raises(pdg.PdgError) as e:
        pdg.pdg_log_v_noalloc(s.ctx, out.data_ptr())
    assert e.value.code == pdg.PDG_ECAPACITY
    assert not out.cpu().numpy().any()
    s.primal_phase()
    s.close()
