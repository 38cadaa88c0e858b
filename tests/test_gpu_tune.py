"""Launch-parameter tuner (``-m gpu``): tuning leaves the chain as it was, the
dual's tiling changes no result, and every setting of the tiling and of the hub
split samples the oracle's conditionals (teacher-forced)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from paper_1611_06684_amd import workloads as W
from tests.test_gpu_parity import _hub_graph, _random_state, teacher_forced

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["grid_q4_C64", "grid_q2_C8", "hubs_C32", "hubs_z_C32"])
def test_tune_keeps_the_chain(case):
    from paper_1611_06684_amd import pdg
    from paper_1611_06684_amd.pdg import Sampler
    model, C = {"grid_q4_C64": (W.table_grid(60, 50, 4, seed=1), 64),
                "grid_q2_C8": (W.table_grid(80, 70, 2, seed=2), 8),
                "hubs_C32": (_hub_graph(700, [2, 3, 5], 4, 9), 32),
                "hubs_z_C32": (_hub_graph(500, [8], 2, 13), 32)}[case]
    a = Sampler(model, C, seed=5, burn_in=1)
    b = Sampler(model, C, seed=5, burn_in=1)
    for s in (a, b):
        s.init()
        s.sweep(3)
    tun = pdg.pdg_tune(a.ctx, 3)
    print(f"  {case}: {tun.as_dict()}", flush=True)
    assert a.t == b.t
    assert np.array_equal(a.state().cpu().numpy(), b.state().cpu().numpy())
    ca, na = a.counts()
    cb, nb = b.counts()
    assert na == nb and np.array_equal(ca, cb)
    got = pdg.pdg_get_tuning(a.ctx)
    assert (got.dual_edges_per_wave, got.hub_threshold) == (tun.dual_edges_per_wave, tun.hub_threshold)
    if not case.startswith("hubs"):  # the tiling changes no result; the hub split may round differently
        for s in (a, b):
            s.sweep(4)
        assert np.array_equal(a.state().cpu().numpy(), b.state().cpu().numpy())
    a.close()
    b.close()


def test_every_setting_samples_the_oracle():
    from paper_1611_06684_amd import pdg
    from paper_1611_06684_amd.pdg import Sampler
    for model, C in [(_hub_graph(700, [2, 3, 5], 4, 9), 32), (_hub_graph(600, [2], 2, 10), 8),
                     (_hub_graph(900, [4], 3, 8), 100)]:
        s = Sampler(model, C, seed=11)
        dec = oracle.decompose(model)
        for k, (e, thr, piece) in enumerate([(2, 0, 128), (8, 128, 64), (4, 512, 256), (8, 256, 32),
                                             (2, 64, 4096)]):
            tun = pdg.pdg_tuning(dual_edges_per_wave=e, binary_groups_per_wave=e, hub_threshold=thr,
                                 hub_piece=piece, dual_ms=-1, primal_ms=-1)
            pdg.pdg_set_tuning(s.ctx, tun)
            x_in = _random_state(model, C, 40 + k)
            r = teacher_forced(s, model, dec, 11, x_in, 3 + k)
            print(f"  C={C} e={e} thr={thr} piece={piece}: {r}", flush=True)
            assert r["bad_dual"] == 0 and r["bad_x"] == 0, r
        bad = pdg.pdg_tuning(dual_edges_per_wave=3, binary_groups_per_wave=4, hub_threshold=256,
                             hub_piece=128, dual_ms=-1, primal_ms=-1)
        with pytest.raises(pdg.PdgError) as ex:
            pdg.pdg_set_tuning(s.ctx, bad)
        assert ex.value.code == pdg.PDG_EINVAL
        s.close()
