"""Learned block proposal on the GPU against the FP64 oracle of Sec. 5.4
blocking (``-m gpu``), through the C ABI.

Bars.  Cut duals, proposals, acceptances and new states: bit-exact except
flagged draws (uniform within 1e-6 of p(theta = 0) for a dual or of sigmoid(l)
for a proposal bit, log u within 1e-9 of the log acceptance ratio), which must
be rare (a proposal row holds 64 draws, so about 1.3e-4 of rows are flagged).  Fields: FP64, within 1e-12 (1 + |f|) (the same sums in
another order).  Network: each layer teacher-forced from the GPU's previous
layer; a layer's FP32 accumulation of K products differs from FP64 by at most
gamma_K sum |w a| (gamma_K = K u / (1 - K u), u = 2^-24), so a BF16 activation
may land one BF16 step away where the exact value sits that close to a
rounding midpoint; logits within gamma_{K+2} (sum |w h| + |b| + |residual|).
Gradients: from the GPU's own BF16 matrices, each FP32 sum over R rows within
gamma_R of the sum of magnitudes.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import block_oracle as B
from oracle import oracle
from paper_1611_06684_amd import workloads as W

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gamma(k):
    return k * U / (1 - k * U)


def _bf16_of_bits(a):
    return (np.asarray(a).astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _params(seed):
    from paper_1611_06684_amd import pdg_block as pb
    rng = np.random.default_rng(seed)
    w = np.zeros(pb.MLP_PARAMS, np.float32)
    for name, shp in pb.SHAPE.items():
        std = np.sqrt(2.0 / shp[-1]) if name.startswith("W") else 0.1
        w[pb.OFF[name]:pb.OFF[name] + int(np.prod(shp))] = rng.normal(0, std, size=shp).ravel()
    return w


def _unpack(w):
    """Oracle parameters: BF16 weight values, FP32 bias values, as float64."""
    from paper_1611_06684_amd import pdg_block as pb
    out = {}
    for name, shp in pb.SHAPE.items():
        v = w[pb.OFF[name]:pb.OFF[name] + int(np.prod(shp))].reshape(shp).astype(np.float64)
        out[name] = B.bf16(v) if name.startswith("W") else v
    return out


def _device_params(w):
    import torch
    from paper_1611_06684_amd import pdg_block as pb
    w32 = torch.as_tensor(w, device="cuda")
    wbf = torch.as_tensor(pb.bf16_bits(w).view(np.int16), device="cuda")
    return w32, wbf


def _layer_check(got_bits, pre_exact, mag, K, name):
    """got: GPU BF16 activations; pre_exact: FP64 pre-activation from the GPU's
    previous layer; mag: sum |w a| + |b| per entry."""
    got = _bf16_of_bits(got_bits)
    want = B.bf16(np.maximum(pre_exact, 0.0))
    bad = got != want
    if bad.any():
        # allowed only where the exact value is within the accumulation bound of
        # a BF16 rounding midpoint (or of 0 for the ReLU)
        lo = B.bf16(np.maximum(pre_exact - _gamma(K + 1) * mag, 0.0))
        hi = B.bf16(np.maximum(pre_exact + _gamma(K + 1) * mag, 0.0))
        ok = (got == lo) | (got == hi)
        assert ok[bad].all(), (name, np.argwhere(bad & ~ok)[:5])
    _say(f"  {name}: {int(bad.sum())} of {bad.size} one BF16 step off (at a midpoint)")
    return int(bad.sum())


@pytest.mark.parametrize("rows", [200, 64, 1])
def test_mlp_forward_matches_oracle(rows):
    import torch
    from paper_1611_06684_amd import pdg_block as pb
    w = _params(1)
    P = _unpack(w)
    w32, wbf = _device_params(w)
    rng = np.random.default_rng(2)
    X = np.concatenate([rng.normal(0, 1.5, (rows, 64)), rng.integers(0, 2, (rows, 32))], 1)
    Xb = B.bf16(X)
    xin = torch.as_tensor(pb.bf16_bits(Xb).view(np.int16), device="cuda")
    lg = torch.zeros((rows, 64), dtype=torch.float32, device="cuda")
    h1 = torch.zeros((rows, 256), dtype=torch.int16, device="cuda")
    h2 = torch.zeros((rows, 256), dtype=torch.int16, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    pb.pdg_mlp_forward(wbf.data_ptr(), w32.data_ptr(), rows, xin.data_ptr(), lg.data_ptr(),
                       h1.data_ptr(), h2.data_ptr(), st)
    torch.cuda.synchronize()
    H1 = _bf16_of_bits(h1.cpu().numpy().view(np.uint16))
    H2 = _bf16_of_bits(h2.cpu().numpy().view(np.uint16))
    L = lg.cpu().numpy().astype(np.float64)
    pre1 = Xb @ P["W1"].T + P["b1"]
    _layer_check(h1.cpu().numpy().view(np.uint16), pre1, np.abs(Xb) @ np.abs(P["W1"]).T + np.abs(P["b1"]),
                 96, "H1")
    pre2 = H1 @ P["W2"].T + P["b2"]
    _layer_check(h2.cpu().numpy().view(np.uint16), pre2, np.abs(H1) @ np.abs(P["W2"]).T + np.abs(P["b2"]),
                 256, "H2")
    want = H2 @ P["W3"].T + P["b3"] + Xb[:, :64]
    mag = np.abs(H2) @ np.abs(P["W3"]).T + np.abs(P["b3"]) + np.abs(Xb[:, :64])
    assert (np.abs(L - want) <= _gamma(258) * mag + 1e-30).all(), np.abs(L - want).max()
    # the whole oracle forward agrees closely too (not teacher-forced)
    _, _, Lo = B.mlp_forward(P, Xb)
    _say(f"  rows {rows}: max |logit - oracle| {np.abs(L - Lo).max():.3g}")
    # without h1 / h2 outputs the logits are the same
    lg2 = torch.zeros_like(lg)
    pb.pdg_mlp_forward(wbf.data_ptr(), w32.data_ptr(), rows, xin.data_ptr(), lg2.data_ptr(),
                       0, 0, st)
    torch.cuda.synchronize()
    assert torch.equal(lg, lg2)


def test_mlp_backward_and_adam_match_oracle():
    import torch
    from paper_1611_06684_amd import pdg_block as pb
    rows = 300
    w = _params(3)
    P = _unpack(w)
    w32, wbf = _device_params(w)
    rng = np.random.default_rng(4)
    Xb = B.bf16(np.concatenate([rng.normal(0, 1.5, (rows, 64)), rng.integers(0, 2, (rows, 32))], 1))
    T = rng.integers(0, 2, (rows, 64)).astype(np.uint8)
    dev = "cuda"
    xin = torch.as_tensor(pb.bf16_bits(Xb).view(np.int16), device=dev)
    tg = torch.as_tensor(T, device=dev)
    lg = torch.zeros((rows, 64), dtype=torch.float32, device=dev)
    h1 = torch.zeros((rows, 256), dtype=torch.int16, device=dev)
    h2 = torch.zeros((rows, 256), dtype=torch.int16, device=dev)
    grad = torch.full((pb.MLP_PARAMS,), float("nan"), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    nbytes = pb.pdg_mlp_backward_workspace(rows)
    work = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    pb.pdg_mlp_forward(wbf.data_ptr(), w32.data_ptr(), rows, xin.data_ptr(), lg.data_ptr(),
                       h1.data_ptr(), h2.data_ptr(), st)
    pb.pdg_mlp_backward(wbf.data_ptr(), rows, xin.data_ptr(), h1.data_ptr(), h2.data_ptr(),
                        lg.data_ptr(), tg.data_ptr(), grad.data_ptr(), loss.data_ptr(),
                        work.data_ptr(), nbytes, st)
    torch.cuda.synchronize()
    H1 = _bf16_of_bits(h1.cpu().numpy().view(np.uint16))
    H2 = _bf16_of_bits(h2.cpu().numpy().view(np.uint16))
    L = lg.cpu().numpy().astype(np.float64)
    wk = work.cpu().numpy()
    a = lambda k: (k + 255) // 256 * 256
    dL = _bf16_of_bits(wk[:rows * 128].view(np.uint16).reshape(rows, 64))
    o2 = a(rows * 128)
    dH2 = _bf16_of_bits(wk[o2:o2 + rows * 512].view(np.uint16).reshape(rows, 256))
    o1 = o2 + a(rows * 512)
    dH1 = _bf16_of_bits(wk[o1:o1 + rows * 512].view(np.uint16).reshape(rows, 256))
    g = grad.cpu().numpy().astype(np.float64)
    # dl = (sigmoid(l) - t) / R in FP32 on the GPU: within a few FP32 ulps
    dl = (1.0 / (1.0 + np.exp(-L)) - T) / rows
    assert (np.abs(dL - dl) <= 2.0 ** -8 * np.abs(dl) + 4 * U * (1.0 / rows) + 1e-30).all()
    # masked products from the GPU's own matrices
    pre = (dL @ P["W3"]) * (H2 > 0)
    mag = (np.abs(dL) @ np.abs(P["W3"])) * (H2 > 0)
    assert (np.abs(dH2 - B.bf16(pre)) <= 2.0 ** -7 * np.abs(pre) + _gamma(64) * mag + 1e-30).all()
    pre = (dH2 @ P["W2"]) * (H1 > 0)
    mag = (np.abs(dH2) @ np.abs(P["W2"])) * (H1 > 0)
    assert (np.abs(dH1 - B.bf16(pre)) <= 2.0 ** -7 * np.abs(pre) + _gamma(256) * mag + 1e-30).all()
    gam = _gamma(rows + 2)

    def check(name, want, mag):
        got = g[pb.OFF[name]:pb.OFF[name] + want.size].reshape(want.shape)
        err = np.abs(got - want)
        assert (err <= gam * mag + 1e-30).all(), (name, err.max(), (gam * mag).max())

    check("W3", dL.T @ H2, np.abs(dL).T @ np.abs(H2))
    check("W2", dH2.T @ H1, np.abs(dH2).T @ np.abs(H1))
    check("W1", dH1.T @ Xb, np.abs(dH1).T @ np.abs(Xb))
    check("b3", dL.sum(0), np.abs(dL).sum(0))
    check("b2", dH2.sum(0), np.abs(dH2).sum(0))
    check("b1", dH1.sum(0), np.abs(dH1).sum(0))
    lo = B.mlp_loss(L, T)
    assert abs(float(loss.cpu()[0]) - lo) < 1e-5 * lo
    # and against the full FP64 backward of the oracle (no teacher forcing): close
    go = B.mlp_backward(P, Xb, H1, H2, L, T)
    rel = np.abs(g[pb.OFF["W2"]:pb.OFF["W2"] + 65536] - go["W2"].ravel()).max() / np.abs(go["W2"]).max()
    _say(f"  W2 gradient vs oracle backward: max relative difference {rel:.3g}")
    assert rel < 2e-2
    # Adam step 3 from given moments
    m0 = rng.normal(0, 1e-3, pb.MLP_PARAMS).astype(np.float32)
    v0 = np.abs(rng.normal(0, 1e-6, pb.MLP_PARAMS)).astype(np.float32)
    gm = torch.as_tensor(m0, device=dev)
    gv = torch.as_tensor(v0, device=dev)
    pb.pdg_mlp_adam(w32.data_ptr(), grad.data_ptr(), gm.data_ptr(), gv.data_ptr(), 3, 1e-3, 0.9,
                    0.999, 1e-8, wbf.data_ptr(), st)
    torch.cuda.synchronize()
    # the hyperparameters as the GPU holds them (FP32 values)
    f32 = lambda v: float(np.float32(v))
    w_new, _, _ = B.adam(w.astype(np.float64), g, m0.astype(np.float64), v0.astype(np.float64), 3,
                         f32(1e-3), f32(0.9), f32(0.999), f32(1e-8))
    got = w32.cpu().numpy().astype(np.float64)
    # FP32 arithmetic: a few roundings relative to |w| and to the update's
    # magnitude before the moment m's cancellation (beta1 |m0| + (1-beta1) |g|)
    c1, c2 = 1 / (1 - 0.9 ** 3), 1 / (1 - 0.999 ** 3)
    vh = (0.999 * v0 + 0.001 * g * g) * c2
    upd = 1e-3 * c1 * (0.9 * np.abs(m0) + 0.1 * np.abs(g)) / (np.sqrt(vh) + 1e-8)
    err = np.abs(got - w_new)
    tol = 16 * U * (np.abs(w) + upd) + 1e-12
    assert (err <= tol).all(), (err.max(), np.argmax(err / tol), (err / tol).max())
    assert np.array_equal(wbf.cpu().numpy().view(np.uint16), pb.bf16_bits(w32.cpu().numpy()))


def _grid_model(H, Wd, seed, dtype="f32"):
    return W.table_grid(H, Wd, 2, seed=seed, pair_std=0.5, unary_std=0.5, dtype=dtype)


@pytest.mark.parametrize("H,Wd,C,dtype", [(24, 16, 5, "f32"), (16, 16, 64, "f64"), (8, 24, 33, "f32")])
def test_block_step_matches_oracle(H, Wd, C, dtype):
    """Teacher-forced learned steps: from a random state, cut duals, fields,
    inputs, targets, proposals, acceptances and the new state against the
    oracle (the oracle takes the GPU's duals for the fields and the GPU's logits
    for the proposal), for several step counters."""
    import torch
    from paper_1611_06684_amd import pdg_block as pb
    from paper_1611_06684_amd.pdg import Sampler
    model = _grid_model(H, Wd, 7)
    if dtype == "f64":
        model = W.Model(model.q, model.lam.astype(np.float64), model.src, model.dst,
                        model.Lam.astype(np.float64))
    seed = 13
    s = Sampler(model, C, seed=seed)
    bp = pb.BlockProposal(s, model, H, Wd, init_seed=3)
    blk = B.Blocking(H, Wd, 8)
    dec = oracle.decompose(model)
    rng = np.random.default_rng(8)
    nb, rows = blk.nb, blk.nb * C
    tot = dict(flag_rows=0, rows=0, dflag=0, duals=0, accepted=0)
    for step in range(1, 5):
        x = rng.integers(0, 2, size=(model.n, C)).astype(np.uint8)
        s.set_state(torch.as_tensor(x, device=s.dev))
        prop = torch.zeros((rows, 64), dtype=torch.uint8, device=s.dev)
        acc = torch.zeros(rows, dtype=torch.uint8, device=s.dev)
        flag = torch.zeros(rows, dtype=torch.uint8, device=s.dev)
        fields = torch.zeros((rows, 64), dtype=torch.float64, device=s.dev)
        tgt = torch.zeros((rows, 64), dtype=torch.uint8, device=s.dev)
        bp.step(prop=prop, acc=acc, flag=flag, fields=fields, target=tgt)
        th_g = torch.zeros((model.m, C), dtype=torch.uint8, device=s.dev)
        pb.pdg_blk_get_cut_duals(bp.blk, th_g.data_ptr(), s.ctx)
        th_g = th_g.cpu().numpy()
        x_g = s.state().cpu().numpy()
        th_o, dfl = B.cut_duals(model, dec, blk, x, seed, step)
        assert ((th_g != th_o) & (dfl == 0)).sum() == 0
        assert not th_g[~blk.cut].any()
        tot["dflag"] += int(dfl[blk.cut].sum())
        tot["duals"] += int(blk.cut.sum()) * C
        f_o, internal = B.block_fields(model, dec, blk, th_g)
        K = B.block_couplings(blk, internal)
        f_g = fields.cpu().numpy().reshape(nb, C, 64)
        assert (np.abs(f_g - f_o) <= 1e-12 * (1 + np.abs(f_o))).all()
        xin = bp.x_in.cpu().numpy().view(np.uint16).reshape(nb, C, 96)
        assert np.array_equal(xin[..., :64], pb.bf16_bits(f_g.astype(np.float32)))
        X_o = B.mlp_inputs(blk, f_o, th_g).reshape(nb, C, 96)
        assert np.array_equal(_bf16_of_bits(xin[..., 64:]), X_o[..., 64:])
        assert np.array_equal(tgt.cpu().numpy().reshape(nb, C, 64),
                              np.transpose(x[blk.nodes], (0, 2, 1)))
        lg = bp.logits.cpu().numpy().reshape(nb, C, 64)
        x_o, acc_o, fl_o, xp_o = B.mh_step(blk, x, f_g, K, lg, seed, step)
        fl_g = flag.cpu().numpy().reshape(nb, C).astype(bool)
        assert np.array_equal(fl_g, fl_o), "flags differ"
        ok = ~fl_o
        assert np.array_equal(prop.cpu().numpy().reshape(nb, C, 64)[ok], xp_o[ok])
        assert np.array_equal(acc.cpu().numpy().reshape(nb, C).astype(bool)[ok], acc_o[ok])
        # the new state: every block whose draw is unflagged
        for b in range(nb):
            for c in np.flatnonzero(ok[b]):
                assert np.array_equal(x_g[blk.nodes[b], c], x_o[blk.nodes[b], c]), (b, c)
        tot["flag_rows"] += int(fl_o.sum())
        tot["rows"] += rows
        tot["accepted"] += int(acc_o.sum())
    _say(f"  {H}x{Wd} C={C} {dtype}: {tot}")
    assert tot["flag_rows"] <= max(2e-3 * tot["rows"], 3)
    assert tot["dflag"] <= max(1e-5 * tot["duals"], 2)
    s_info = pb.pdg_blk_info(bp.blk, s.ctx)
    assert s_info[0] == 4 and s_info[3] == 4 * rows
    bp.close()
    s.close()


def test_learned_steps_keep_the_marginals():
    """A chain alternating learned steps (untrained network) with plain sweeps
    and a chain of plain sweeps only have the same marginals on a 16 x 16 grid
    with couplings J ~ U(0, 0.35) (batch-means standard errors, |z| < 4.5 over
    the 256 nodes)."""
    import torch
    from paper_1611_06684_amd import pdg, pdg_block as pb
    from paper_1611_06684_amd.pdg import Sampler
    from tests import brute
    rng = np.random.default_rng(21)
    src, dst = W.grid_edges(16, 16)
    model = W.ising_model(src, dst, rng.uniform(0, 0.35, src.shape[0]), rng.normal(0, 0.3, 256), 256,
                          "f32")
    C = 128
    est = {}
    for learned in (False, True):
        s = Sampler(model, C, seed=31 + learned, burn_in=0)
        bp = pb.BlockProposal(s, model, 16, 16, init_seed=5) if learned else None
        s.init()
        for _ in range(100):
            if bp:
                bp.step()
            s.sweep(1)
        batches = []
        cnt = torch.zeros((256, 2), dtype=torch.int32, device=s.dev)
        for b in range(30):
            s.reset_marginals()
            for _ in range(40):
                if bp:
                    bp.step()
                s.sweep(1)
            n = pdg.pdg_get_counts(s.ctx, cnt.data_ptr())
            batches.append(cnt.cpu().numpy()[:, 1] / n)
        est[learned] = brute.batch_means(np.array(batches))
        if bp:
            _say(f"  acceptance {bp.accept_rate():.4f}")
            bp.close()
        s.close()
    (m0, s0), (m1, s1) = est[False], est[True]
    z = np.abs(m0 - m1) / np.sqrt(s0 ** 2 + s1 ** 2)
    _say(f"  max |z| {z.max():.2f}")
    assert (z < 4.5).all()


def test_full_size_learned_step_sampled():
    """The learned-proposal workload at full size (512 x 512 binary grid, J ~
    U(0, 0.35), h ~ N(0, 0.3), 8 x 8 blocks, 128 chains) in the benchmark's
    launch configuration: one learned step from a state of the plain chain;
    every cut dual against the oracle, and for 24 sampled blocks (corners and
    edges included) the proposals, acceptances and new states."""
    import torch
    from paper_1611_06684_amd import learned as Lw
    from paper_1611_06684_amd import pdg_block as pb
    from paper_1611_06684_amd.pdg import Sampler
    side, C, seed = 512, 128, 0
    model = Lw.grid_model(side, seed=0)
    s = Sampler(model, C, seed=seed)
    s.init()
    s.sweep(20)
    bp = pb.BlockProposal(s, model, side, side, init_seed=0)
    x = s.state().cpu().numpy()
    rows = bp.rows
    prop = torch.zeros((rows, 64), dtype=torch.uint8, device=s.dev)
    acc = torch.zeros(rows, dtype=torch.uint8, device=s.dev)
    flag = torch.zeros(rows, dtype=torch.uint8, device=s.dev)
    bp.step(prop=prop, acc=acc, flag=flag)
    th_g = torch.zeros((model.m, C), dtype=torch.uint8, device=s.dev)
    pb.pdg_blk_get_cut_duals(bp.blk, th_g.data_ptr(), s.ctx)
    th_g = th_g.cpu().numpy()
    x_g = s.state().cpu().numpy()
    lg = bp.logits.cpu().numpy()
    prop = prop.cpu().numpy()
    acc = acc.cpu().numpy().astype(bool)
    fl_g = flag.cpu().numpy().astype(bool)
    bp.close()
    s.close()
    blk = B.Blocking(side, side, 8)
    dec = oracle.decompose(model)
    th_o, dfl = B.cut_duals(model, dec, blk, x, seed, 1)
    assert ((th_g != th_o) & (dfl == 0)).sum() == 0
    n_dflag = int(dfl[blk.cut].sum())
    _say(f"  cut duals: {int(blk.cut.sum()) * C} draws, flagged {n_dflag}")
    assert n_dflag <= max(1e-5 * blk.cut.sum() * C, 3)
    f_o, internal = B.block_fields(model, dec, blk, th_g)
    K = B.block_couplings(blk, internal)
    rng = np.random.default_rng(3)
    blocks = np.unique(np.concatenate([[0, 63, 4032, 4095, 64, 127], rng.choice(blk.nb, 18,
                                                                                replace=False)]))
    lgb = lg.reshape(blk.nb, C, 64)[blocks]
    x_o, acc_o, fl_o, xp_o = B.mh_step(blk, x, f_o[blocks], K[blocks], lgb, seed, 1, blocks=blocks)
    fl_gb = fl_g.reshape(blk.nb, C)[blocks]
    assert np.array_equal(fl_gb, fl_o)
    ok = ~fl_o
    assert np.array_equal(prop.reshape(blk.nb, C, 64)[blocks][ok], xp_o[ok])
    assert np.array_equal(acc.reshape(blk.nb, C)[blocks][ok], acc_o[ok])
    for j, b in enumerate(blocks):
        for c in np.flatnonzero(ok[j]):
            assert np.array_equal(x_g[blk.nodes[b], c], x_o[blk.nodes[b], c]), (b, c)
    _say(f"  {len(blocks)} blocks x {C} chains: accepted {int(acc_o.sum())}, flagged {int(fl_o.sum())}")
