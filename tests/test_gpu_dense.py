"""The dense gather two ways (``-m gpu``): the field of state 1 of every node of
complete binary graphs given the current duals, by vector FMAs and by FP64
matrix-core products, against each other and against the oracle's node logits
for the same duals (the library's field of state 1 is the logit L(1): base
holds the unary and the duals-free part of every incident factor)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle
from paper_1611_06684_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("C", [8, 16, 5])
def test_dense_fields_mfma_equals_valu_and_oracle(C):
    import torch
    from paper_1611_06684_amd import pdg_block as pb
    from paper_1611_06684_amd.pdg import Sampler
    _, model = W.batched_by_states(3, 2, seed=4, n_min=50, n_max=200, dense_n=300)[0]
    s = Sampler(model, C, seed=2)
    s.init()
    s.sweep(2)
    s.dual_phase()
    nd = 600  # the two dense graphs come first
    nodes = torch.arange(nd, dtype=torch.int32, device=s.dev)
    outs = []
    for method in (0, 1):
        out = torch.full((nd, C), float("nan"), dtype=torch.float64, device=s.dev)
        pb.pdg_dense_fields(s.ctx, nd, nodes.data_ptr(), method, out.data_ptr())
        s.sync()
        outs.append(out.cpu().numpy())
    th = s.duals(s.uids).cpu().numpy().view(np.uint64)
    s.primal_phase()
    s.close()
    v, m = outs
    assert np.isfinite(v).all() and np.isfinite(m).all()
    # the same 299 terms per node added in other orders: a few ulps of the
    # largest partial sum
    scale = np.abs(v).max() + np.abs(model.lam).max() + 1.0
    assert np.abs(v - m).max() <= 300 * 4 * 2.0 ** -53 * 300 * scale
    dec = oracle.decompose(model)
    for c in range(C):
        L = oracle.all_logits(model, dec, np.ascontiguousarray(th[:, c]))
        np.testing.assert_allclose(m[:, c], L[:nd, 1], rtol=0, atol=1e-9 * scale)
        np.testing.assert_allclose(v[:, c], L[:nd, 1], rtol=0, atol=1e-9 * scale)
