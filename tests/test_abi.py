"""CPU checks of the C ABI: the library loads, exports every function that
include/pdg.h declares, and rejects bad arguments before touching a GPU."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1611_06684_amd import pdg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="pdg.h"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^(?:pdg_status|const char \*)\s*(pdg_\w+)\(", txt, re.M)))


def test_header_and_binding_agree():
    declared = _declared()
    assert len(declared) >= 20
    assert sorted(pdg.EXPORTS) == declared
    from paper_1611_06684_amd import pdg_block, rates
    assert sorted(pdg_block.EXPORTS) == _declared("pdg_block.h")
    assert sorted(rates.EXPORTS) == _declared("pdg_rates.h")


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(pdg.LIB_PATH)
    for name in _declared() + _declared("pdg_block.h") + _declared("pdg_rates.h"):
        assert hasattr(L, name), name


def test_packed_network_layout_matches_header():
    from paper_1611_06684_amd import pdg_block as pb
    txt = open(os.path.join(ROOT, "include", "pdg_block.h")).read()
    for name, off in pb.OFF.items():
        key = "PDG_MLP_OFF_" + name.upper()
        assert re.search(key + r" = (\d+)", txt).group(1) == str(off)
    total = 0
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert pb.OFF[name] == total
        total += int(np.prod(pb.SHAPE[name]))
    assert total == pb.MLP_PARAMS


def test_params_layout():
    for q in range(2, 9):
        D = (q - 1) ** 2
        assert pdg.pdg_params_layout(q) == (8 + 16 * D + 16 * (q - 1), 0, 8, 8 + 8 * D,
                                            8 + 16 * D)
    with pytest.raises(pdg.PdgError) as e:
        pdg.pdg_params_layout(9)
    assert e.value.code == pdg.PDG_EINVAL


@pytest.mark.parametrize("field,value", [("n_chains", 0), ("q_max", 1), ("q_max", 9),
                                         ("edge_capacity", 0), ("precision", 7),
                                         ("reserved", 1), ("burn_in", -1)])
def test_create_rejects_bad_config(field, value):
    cfg = pdg.pdg_config(seed=0, n_chains=4, q_max=4, node_capacity=10, edge_capacity=10,
                         precision=0, reserved=0, burn_in=0)
    setattr(cfg, field, value)
    with pytest.raises(pdg.PdgError) as e:
        pdg.pdg_create(cfg, 0, 0)
    assert e.value.code == pdg.PDG_EINVAL


def test_null_context_is_an_error():
    for fn in (pdg.pdg_sweep, pdg.pdg_init_chains, pdg.pdg_sync):
        with pytest.raises(pdg.PdgError):
            fn(None) if fn is not pdg.pdg_sweep else fn(None, 1)
