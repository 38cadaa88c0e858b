"""GPU path vs the FP64 oracle, through the C ABI (``-m gpu``).

Parity bar (the sampler's floating point decides integers):
  * init and every *unflagged* draw bit-exact; a draw is flagged when its
    uniform lies within 1e-6 of a CDF boundary computed by the oracle in FP64;
  * flagged draws may differ and must be fewer than 1e-5 of all draws;
  * FP64 contexts (FP64 exp in the node draw) match free-running trajectories
    and marginal counters exactly;
  * marginals agree with enumeration within 3 batch-means standard errors.
Teacher forcing: both sides start a sweep from the same x; the oracle's primal
phase is fed the GPU's duals, so one flagged dual cannot cascade.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1611_06684_amd import workloads as W
from tests import brute

pytestmark = pytest.mark.gpu

FLAG_BUDGET = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sampler(model, C, seed, **kw):
    from paper_1611_06684_amd.pdg import Sampler
    return Sampler(model, C, seed=seed, **kw)


def _random_state(model, C, seed):
    rng = np.random.default_rng(seed)
    return (rng.random((model.n, C)) * model.q[:, None]).astype(np.uint8)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _histogram(x, q_max):
    """Per node, how many chains are in each state: int64 [n][q_max]."""
    return np.stack([(x == a).sum(axis=1) for a in range(q_max)], axis=1).astype(np.int64)


def teacher_forced(s, model, dec, seed, x_in, t):
    """One sweep t on GPU and oracle from x_in.  Returns a dict of counts.
    The marginal counters (counting on: t > burn-in) must grow by exactly the
    per-node histogram of the new states, which are checked against the oracle
    draw by draw: this covers the counting code of every primal shape."""
    import torch
    s.t = t - 1
    s.set_state(torch.as_tensor(x_in, device=s.dev))
    cnt0, n0 = s.counts()
    s.dual_phase()
    th_g = _u64(s.duals(s.uids))
    s.primal_phase()
    x_g = s.state().cpu().numpy()
    cnt1, n1 = s.counts()
    assert n1 - n0 == x_in.shape[1], (n0, n1)
    assert np.array_equal(cnt1 - cnt0, _histogram(x_g, s.q_max)), "counter delta != histogram"
    uid = _u64(s.uids)
    th_o, dflag, _, _ = oracle.sweep(model, dec, uid, seed, t, x_in)
    x_o, pflag = oracle.primal_phase(model, dec, seed, t, th_g)
    dmis = th_g ^ th_o
    bad_dual = int(np.count_nonzero(dmis & ~dflag))
    xmis = x_g != x_o
    bad_x = int(np.count_nonzero(xmis & (pflag == 0)))
    D = (model.q[model.src] - 1) * (model.q[model.dst] - 1)
    n_draws = int(D.sum()) * x_in.shape[1] + model.n * x_in.shape[1]
    n_flag = int(sum(bin(int(v)).count("1") for v in dflag.ravel() if v)) + int(pflag.sum())
    return dict(bad_dual=bad_dual, bad_x=bad_x, dual_mis=int(np.count_nonzero(dmis)),
                x_mis=int(xmis.sum()), flagged=n_flag, draws=n_draws)


def _models():
    yield "tiny_ising_4x4_f64_C1", W.ising_grid(4, 4, seed=0), 1
    yield "grid_37x29_q4_f32_C64", W.table_grid(37, 29, 4, seed=1), 64
    yield "grid_20x23_q3_f32_C32", W.table_grid(20, 23, 3, seed=2, pair_std=0.6), 32
    yield "random_mixed_q235_f32_C5", W.random_graph(300, 900, [2, 3, 5], seed=3, dtype="f32"), 5
    yield "random_mixed_q2to7_f64_C17", W.random_graph(200, 500, [2, 4, 7], seed=4), 17
    yield "grid_16x16_q2_f32_C100", W.table_grid(16, 16, 2, seed=5, pair_std=1.0), 100
    yield "ising_10x10_f64_C13", W.ising_grid(10, 10, seed=6, J_half_range=0.8), 13
    yield "chung_lu_4096_q8_f32_C32", W.chung_lu(4096, 8, seed=7), 32
    # 33+ chains with large q_max: two-load LDS staging, mixed and uniform q
    yield "random_mixed_q678_f32_C40", W.random_graph(400, 1600, [6, 7, 8], seed=11, dtype="f32"), 40
    yield "grid_18x17_q6_f64_C64", W.table_grid(18, 17, 6, seed=12, dtype="f64"), 64
    # hubs: nodes with more incidences than a quad kernel takes (split into pieces)
    # a batch of independent uneven graphs (mixed q per graph, two dense binary ones)
    yield "batch_30_f32_C8", W.batched_uneven(30, 2, seed=1, n_min=20, n_max=300, dense_n=40), 8
    # the same batch as one model per state count (uniform-q kernels, records of that q)
    for q, g in W.group_by_states(W.batched_uneven(30, 2, seed=1, n_min=20, n_max=300,
                                                   dense_n=40)):
        yield f"batch_30_q{q}_f32_C8", g, 8
    yield "hubs_q4_f32_C64", _hub_graph(900, [4], 3, 8), 64
    yield "hubs_mixed_q235_f32_C32", _hub_graph(700, [2, 3, 5], 4, 9), 32
    yield "hubs_q2_f32_C100", _hub_graph(600, [2], 2, 10), 100
    # hubs with 16 or fewer chains: 64 / LPI lane groups share a piece's records
    yield "hubs_q2_f32_C1", _hub_graph(600, [2], 2, 10), 1
    yield "hubs_mixed_q235_f32_C5", _hub_graph(700, [2, 3, 5], 4, 9), 5
    yield "hubs_q4_f32_C16", _hub_graph(900, [4], 3, 8), 16
    # binary records with 16 and 3 chains (E item groups per wave, ragged)
    yield "grid_21x19_q2_f32_C16", W.table_grid(21, 19, 2, seed=14), 16
    yield "ising_9x7_f64_C3", W.ising_grid(9, 7, seed=15), 3
    # 2-16 chains with lanes of absent chains in every item, mixed and uniform
    # q up to 8 (staged primal with several loads per step, gathered dual words)
    yield "random_mixed_q258_f32_C9", W.random_graph(250, 600, [2, 5, 8], seed=21, dtype="f32"), 9
    yield "random_mixed_q36_f64_C12", W.random_graph(250, 600, [3, 6], seed=22), 12
    yield "random_q7_f32_C15", W.random_graph(200, 500, [7], seed=23, dtype="f32"), 15
    yield "random_q4_f32_C7", W.random_graph(300, 700, [4], seed=24, dtype="f32"), 7
    yield "random_mixed_q23_f32_C2", W.random_graph(300, 700, [2, 3], seed=25, dtype="f32"), 2
    # q_max 8 with 8 chains: a step's records do not fit the piece kernel's
    # LDS chunk, so hubs stay with the quad kernel
    yield "hubs_q8_f32_C8", _hub_graph(500, [8], 2, 13), 8
    # 17..32 chains with q_max >= 6: chain-major dual words, table-based primal
    # and hub pieces; uniform and mixed q (entries of smaller tables, binary
    # nodes), ragged chain counts
    yield "random_q6_f32_C24", W.random_graph(300, 900, [6], seed=26, dtype="f32"), 24
    yield "random_mixed_q267_f32_C29", W.random_graph(300, 800, [2, 6, 7], seed=27, dtype="f32"), 29
    yield "hubs_q8_f32_C32", _hub_graph(500, [8], 2, 13), 32
    yield "hubs_mixed_q68_f64_C20", _hub_graph(600, [6, 8], 3, 16, np.float64), 20


def _hub_graph(n, qs, n_hubs, seed, dtype=np.float32):
    """n nodes with q uniform from qs; hub h (h < n_hubs) is joined to 300 + 130 h
    other nodes (as src or dst alternately), plus 2 n random edges; tables
    N(0, 0.5), entries beyond a node's q zero, unaries N(0, 1), FP32 (or dtype)."""
    rng = np.random.default_rng(seed)
    q = rng.choice(np.asarray(qs), size=n).astype(np.int32)
    src, dst = [], []
    for h in range(n_hubs):
        others = rng.choice(np.setdiff1d(np.arange(n), [h]), size=300 + 130 * h, replace=False)
        for k, o in enumerate(others):
            src.append(h if k % 2 == 0 else o)
            dst.append(o if k % 2 == 0 else h)
    a = rng.integers(0, n, 2 * n)
    b = (a + 1 + rng.integers(0, n - 1, 2 * n)) % n
    src = np.concatenate([np.asarray(src), a]).astype(np.int32)
    dst = np.concatenate([np.asarray(dst), b]).astype(np.int32)
    qm = int(max(qs))
    Lam = rng.normal(0.0, 0.5, size=(len(src), qm, qm))
    lam = rng.normal(0.0, 1.0, size=(n, qm))
    ar = np.arange(qm)
    Lam[np.broadcast_to(ar[None, :, None] >= q[src][:, None, None], Lam.shape)] = 0.0
    Lam[np.broadcast_to(ar[None, None, :] >= q[dst][:, None, None], Lam.shape)] = 0.0
    lam[ar[None, :] >= q[:, None]] = 0.0
    return W.Model(q, lam.astype(dtype), src, dst, Lam.astype(dtype), f"hubs_{n}")


@pytest.mark.parametrize("name,model,C", list(_models()), ids=[m[0] for m in _models()])
def test_teacher_forced_sweeps(name, model, C):
    _say(f"[teacher-forced] {name} n={model.n} m={model.m} C={C}")
    seed = 11
    s = _sampler(model, C, seed)
    dec = oracle.decompose(model)
    tot = dict(flagged=0, draws=0)
    for k, t in enumerate((1, 2, 7, 123457)):
        x_in = _random_state(model, C, 100 + k)
        r = teacher_forced(s, model, dec, seed, x_in, t)
        _say(f"  t={t} {r}")
        assert r["bad_dual"] == 0, r
        assert r["bad_x"] == 0, r
        tot["flagged"] += r["flagged"]
        tot["draws"] += r["draws"]
    s.close()
    assert tot["flagged"] <= max(FLAG_BUDGET * tot["draws"], 3), tot



def _log_v_tolerance(model, x, o):
    """Bound on |GPU - oracle| for log V: both add the same N = n + m terms in
    FP64 in different orders (error <= N 2^-53 of the sum of magnitudes each),
    and the fields L differ by the rounding of two FP64 decompositions
    (1e-13 of that sum is generous)."""
    lam = np.asarray(model.lam, np.float64)
    Lam = np.asarray(model.Lam, np.float64)
    C = x.shape[1]
    lp = np.zeros(C)
    a_abs = np.zeros(C)
    for c in range(C):
        t1 = lam[np.arange(model.n), x[:, c]]
        t2 = Lam[np.arange(model.m), x[model.src, c], x[model.dst, c]]
        lp[c] = t1.sum() + t2.sum()
        a_abs[c] = np.abs(t1).sum() + np.abs(t2).sum()
    s_abs = a_abs + np.abs(o - lp)  # sum_i -log p(x_i | theta) >= 0
    N = model.n + model.m
    return 4 * N * 2.0 ** -53 * s_abs + 1e-13 * s_abs


@pytest.mark.parametrize("name,model,C", list(_models()), ids=[m[0] for m in _models()])
def test_log_v_matches_oracle(name, model, C):
    """Sec. 5.2 estimator between the phases of a teacher-forced sweep: the
    GPU's log V(x, theta) per chain against the oracle's on the same x and the
    GPU's duals, for every kernel shape (hubs, chain blocks, mixed q)."""
    import torch
    seed = 4
    s = _sampler(model, C, seed)
    dec = oracle.decompose(model)
    x_in = _random_state(model, C, 21)
    s.t = 6
    s.set_state(torch.as_tensor(x_in, device=s.dev))
    s.dual_phase()
    g = s.log_v().cpu().numpy()
    th = _u64(s.duals(s.uids))
    o = oracle.log_v(model, dec, th, x_in)
    tol = _log_v_tolerance(model, x_in, o)
    err = np.abs(g - o)
    _say(f"  {name}: max |diff| {err.max():.3g}, max tol {tol.max():.3g}, log V ~ {o.mean():.4g}")
    assert (err <= tol).all(), (err, tol)
    s.primal_phase()
    s.close()


def test_log_v_mean_is_log_z_minus_mutual_information():
    """Sec. 5.2 end to end on the GPU: on a 3x3 Ising model (12 duals, so the
    joint can be enumerated) the average of log V over the sampler's sweeps and
    64 chains equals log Z - I(x; theta) within 4 batch-means standard errors,
    and stays below log Z."""
    import torch
    from tests import brute
    model = W.ising_grid(3, 3, seed=41, J_half_range=0.6)
    dec = oracle.decompose(model)
    X, TH, P = brute.joint(model, dec)
    lp = brute.log_joint(model, X)
    log_Z = lp.max() + np.log(np.exp(lp - lp.max()).sum())
    px, pth = P.sum(axis=1), P.sum(axis=0)
    I = float((P * (np.log(P) - np.log(px)[:, None] - np.log(pth)[None, :])).sum())
    target = log_Z - I
    C = 64
    s = _sampler(model, C, seed=3)
    s.init()
    s.sweep(200)
    nb, per = 40, 100
    means = []
    for b in range(nb):
        acc = torch.zeros(C, dtype=torch.float64, device=s.dev)
        for _ in range(per):
            s.dual_phase()
            acc += s.log_v()
            s.primal_phase()
        means.append(acc.cpu().numpy().mean() / per)
    means = np.array(means)
    m, se = means.mean(), means.std(ddof=1) / np.sqrt(nb)
    _say(f"  mean log V {m:.5f} +- {se:.5f}; log Z - I = {target:.5f}; log Z = {log_Z:.5f}; I = {I:.4f}")
    assert abs(m - target) < 4 * se + 1e-6, (m, se, target)
    assert m < log_Z
    s.close()


def _extreme_model(seed):
    """Mixed-q random graph whose tables include odds ratios near 0 and infinity
    (entries of size 30, so some thresholds saturate at 0 or 2^24) and tables
    with every odds ratio exactly 1 (the dual is a fair coin that carries no
    field), plus nodes without edges."""
    m = W.random_graph(120, 200, [2, 3, 4], seed=seed, pair_std=1.0)
    rng = np.random.default_rng(seed + 1)
    Lam = m.Lam.copy()
    for e in range(m.m):
        qs, qd = int(m.q[m.src[e]]), int(m.q[m.dst[e]])
        if e % 3 == 0:
            Lam[e, :qs, :qd] = rng.choice([-30.0, 30.0], size=(qs, qd))
        elif e % 3 == 1:  # rank one: L(a, b) = r(a) + c(b), every odds ratio 1
            r, c = rng.normal(size=qs), rng.normal(size=qd)
            Lam[e, :qs, :qd] = r[:, None] + c[None, :]
    keep = (m.src < 100) & (m.dst < 100)  # nodes 100..119 keep no edge
    return W.Model(m.q, m.lam, m.src[keep], m.dst[keep], Lam[keep], "extreme")


@pytest.mark.parametrize("C", [3, 20, 64])
def test_degenerate_tables_and_empty_graph(C):
    """Edge cases of the method: saturated and unit odds ratios, isolated nodes,
    and a graph with no edges at all (the primal then draws from the unaries),
    each teacher-forced against the oracle for every kernel shape."""
    for model in (_extreme_model(71), W.Model(*(lambda m: (m.q, m.lam, m.src[:0], m.dst[:0],
                                                           m.Lam[:0]))(W.random_graph(50, 10, [2, 5], seed=72)))):
        s = _sampler(model, C, seed=6)
        dec = oracle.decompose(model)
        x_in = _random_state(model, C, 73)
        r = teacher_forced(s, model, dec, 6, x_in, 9)
        _say(f"  {model.name} m={model.m} C={C}: {r}")
        assert r["bad_dual"] == 0 and r["bad_x"] == 0, r
        s.close()

def test_init_is_bit_exact():
    for model, C, seed in [(W.random_graph(500, 10, [2, 3, 5, 8], seed=1), 37, 5),
                           (W.ising_grid(4, 4), 1, 0), (W.table_grid(30, 30, 4), 64, 2**40 + 3)]:
        s = _sampler(model, C, seed)
        s.init()
        x_g = s.state().cpu().numpy()
        x_o = oracle.init_state(model, C, seed)
        assert (x_g == x_o).all()
        assert s.t == 0
        s.close()


def test_decompose_matches_oracle_conditionals():
    """pdg_decompose (the kernel the insert path runs) against the oracle's
    Theorem parameters: dual thresholds T(y,y') = ceil(p(theta=0|y,y') 2^24 - 1/2)
    and primal fields (all-zero duals, and the per-dual increment beta)."""
    import torch
    from paper_1611_06684_amd import pdg
    rng = np.random.default_rng(9)
    for qm, f64 in [(2, True), (3, False), (4, False), (5, True), (8, False)]:
        m = 3000
        qs = rng.integers(2, qm + 1, size=m).astype(np.int32)
        qd = rng.integers(2, qm + 1, size=m).astype(np.int32)
        dt = np.float64 if f64 else np.float32
        Lam = rng.normal(0, 1.5, size=(m, qm, qm)).astype(dt)
        Lam[:5] *= 8.0  # large odds ratios
        Lam[5:10] *= 1e-7  # near-unit odds ratios
        dev = torch.device("cuda", 0)
        bb, o_sign, o_thr, o_h, o_c = pdg.pdg_params_layout(qm)
        out = torch.zeros(m * bb, dtype=torch.uint8, device=dev)
        tq = [torch.as_tensor(a, device=dev) for a in (qs, qd, Lam)]
        pdg.pdg_decompose(m, qm, tq[0].data_ptr(), tq[1].data_ptr(), tq[2].data_ptr(),
                          1 if f64 else 0, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        blk = out.cpu().numpy().reshape(m, bb)
        D = (qm - 1) ** 2
        sign = blk[:, o_sign:o_sign + 8].copy().view(np.uint64)[:, 0]
        thr = blk[:, o_thr:o_thr + 8 * D].copy().view(np.uint32).reshape(m, D, 2)
        w = 2.0 * blk[:, o_h:o_h + 8 * D].copy().view(np.float64)
        c = blk[:, o_c:o_c + 16 * (qm - 1)].copy().view(np.float64).reshape(m, 2, qm - 1)
        q = np.zeros(2 * m, np.int32)
        q[0::2], q[1::2] = qs, qd
        model = W.Model(q, np.zeros((2 * m, qm)), np.arange(0, 2 * m, 2, dtype=np.int32),
                        np.arange(1, 2 * m, 2, dtype=np.int32), Lam.astype(np.float64))
        dec = oracle.decompose(model)
        n_exact = n_edge = 0
        for e in range(m):
            for a in range(1, qs[e]):
                row_o = dec.rrow[e, a] + sum(dec.par[e, (a - 1) * (qd[e] - 1) + b - 1, 0]
                                             for b in range(1, qd[e]))
                assert abs(row_o - c[e, 0, a - 1]) < 1e-9 * (1 + abs(row_o)), (e, a)
                for b in range(1, qd[e]):
                    d = (a - 1) * (qd[e] - 1) + (b - 1)
                    par = dec.par[e, d]
                    assert abs(w[e, d] - par[3]) < 1e-9 * (1 + abs(par[3]))
                    assert abs(abs(w[e, d]) - par[4]) < 1e-9 * (1 + abs(par[4]))
                    neg = bool((int(sign[e]) >> int(d)) & 1)
                    tp = (int(thr[e, d, 0]) + 1) // 256
                    tm = int(thr[e, d, 1]) // 256
                    assert (int(thr[e, d, 0]) + 1) % 256 == 0 and int(thr[e, d, 1]) % 256 == 0
                    for y in (0, 1):
                        for yp in (0, 1):
                            s1 = (1 - 2 * y) * (-1 if neg else 1)
                            s2 = 1 - 2 * yp
                            T = tp if (s1 > 0 and s2 > 0) else (tm if (s1 < 0 and s2 < 0) else 1 << 23)
                            p0 = 1.0 - oracle.dual_p1(par, y, yp)
                            exact = np.ceil(p0 * 2**24 - 0.5)
                            if T == exact:
                                n_exact += 1
                            else:
                                n_edge += 1
                                frac = p0 * 2**24 - 0.5
                                assert abs(frac - np.round(frac)) < 1e-6, (e, d, y, yp, T, exact)
            for b in range(1, qd[e]):
                col_o = dec.rcol[e, b] + sum(dec.par[e, (a - 1) * (qd[e] - 1) + b - 1, 1]
                                             for a in range(1, qs[e]))
                assert abs(col_o - c[e, 1, b - 1]) < 1e-9 * (1 + abs(col_o)), (e, b)
        _say(f"  q_max={qm}: thresholds exact {n_exact}, on an integer boundary {n_edge}")


def test_decompose_rejects_nonfinite():
    import torch
    from paper_1611_06684_amd import pdg
    dev = torch.device("cuda", 0)
    Lam = torch.zeros((2, 3, 3), dtype=torch.float32, device=dev)
    Lam[1, 2, 1] = float("inf")
    q = torch.full((2,), 3, dtype=torch.int32, device=dev)
    out = torch.zeros(2 * pdg.pdg_params_layout(3)[0], dtype=torch.uint8, device=dev)
    with pytest.raises(pdg.PdgError) as e:
        pdg.pdg_decompose(2, 3, q.data_ptr(), q.data_ptr(), Lam.data_ptr(), 0, out.data_ptr(),
                          torch.cuda.current_stream().cuda_stream)
    assert e.value.code == pdg.PDG_ENONPOS


def test_fp64_free_running_trajectory_and_counts_exact():
    """FP64 context: 2000 free-running sweeps from init, final state and
    marginal counters identical to the oracle's."""
    model = W.ising_grid(6, 5, seed=3, J_half_range=0.7)
    for C in (1, 8, 64):
        s = _sampler(model, C, seed=21, burn_in=100)
        s.init()
        s.sweep(2000)
        x_g = s.state().cpu().numpy()
        import torch
        cnt_g = torch.zeros((model.n, model.q_max), dtype=torch.int32, device=s.dev)
        from paper_1611_06684_amd import pdg
        pdg.pdg_get_counts(s.ctx, cnt_g.data_ptr())
        cnt_g = cnt_g.cpu().numpy().astype(np.uint64)
        dec = oracle.decompose(model)
        x_o = oracle.init_state(model, C, 21)
        cnt_o, nf, nd = oracle.run(model, dec, _u64(s.uids), 21, x_o, 0, 2000, burn_in=100)
        assert (x_g == x_o).all(), C
        assert (cnt_g == cnt_o).all(), C
        s.close()



def test_batched_small_sweeps_match_phase_launches():
    """Small graphs run many sweeps in one launch (k_sweeps, or k_sweeps_lds
    with the state in LDS for the smallest); the trajectory,
    the counters (burn-in crossed inside a batch) and the sweep counter must be
    those of one dual and one primal launch per sweep, bit for bit."""
    import torch
    from paper_1611_06684_amd import pdg
    cases = [(W.random_graph(100, 200, [2, 3, 5], seed=51, dtype="f32"), 5, 7),
             (W.random_graph(60, 120, [8], seed=52, dtype="f32"), 16, 0),
             (W.ising_grid(4, 4, seed=53), 1, 3),
             (W.random_graph(40, 90, [2, 4], seed=54), 12, 20),
             # small enough for the LDS-resident form (q_max <= 5, one thread per item)
             (W.random_graph(30, 50, [2, 3, 4], seed=55, dtype="f32"), 8, 4),
             (W.ising_grid(6, 5, seed=56), 16, 10)]
    for model, C, burn in cases:
        out = []
        for batched in (True, False):
            s = _sampler(model, C, seed=5, burn_in=burn)
            s.init()
            if batched:
                s.sweep(25)
            else:
                for _ in range(25):
                    s.dual_phase()
                    s.primal_phase()
            cnt = torch.zeros((model.n, model.q_max), dtype=torch.int32, device=s.dev)
            samples = pdg.pdg_get_counts(s.ctx, cnt.data_ptr())
            out.append((s.state().cpu().numpy(), cnt.cpu().numpy(), samples, s.t))
            s.close()
        (xa, ca, na, ta), (xb, cb, nb, tb) = out
        _say(f"  {model.name} C={C}: samples {na} / {nb}, t {ta} / {tb}")
        assert ta == tb == 25 and na == nb == C * (25 - burn)
        assert np.array_equal(xa, xb) and np.array_equal(ca, cb)

def test_tiny_marginals_vs_enumeration():
    """Tiny plain workload on the GPU: 4x4 binary grid, FP64, 1 chain, 1e5
    sweeps, seed 0; within 3 batch-means SE of enumeration."""
    import torch
    from paper_1611_06684_amd import pdg
    model = W.ising_grid(4, 4, seed=0)
    exact = brute.exact_marginals(model)
    s = _sampler(model, 1, seed=0)
    s.init()
    s.sweep(10000)
    est = []
    cnt = torch.zeros((model.n, 2), dtype=torch.int32, device=s.dev)
    for b in range(50):
        s.reset_marginals()
        s.sweep(1800)
        n = pdg.pdg_get_counts(s.ctx, cnt.data_ptr())
        est.append(cnt.cpu().numpy() / n)
    mean, se = brute.batch_means(np.array(est))
    z = np.abs(mean[:, 1] - exact[:, 1]) / se[:, 1]
    _say("  z:", np.round(z, 2))
    assert (z < 3).all(), z
    s.close()


def test_edits_then_teacher_forced():
    """Churn on a Chung-Lu graph: remove / insert batches between sweeps; after
    each batch the GPU sweep matches the oracle on the live edge set (by uid)."""
    import torch
    model = W.chung_lu(2048, 5, seed=12)
    C = 32
    seed = 5
    s = _sampler(model, C, seed, edge_capacity=model.m + 2000)
    churn = W.Churn(model.n, 5, model.meta["weights"], seed=13, frac=0.05)
    live_src, live_dst, live_Lam = model.src.copy(), model.dst.copy(), model.Lam.copy()
    live_uid = _u64(s.uids).copy()
    s.init()
    s.sweep(3)
    for rnd in range(4):
        rem, ns, nd, nL = churn.next_batch(live_uid)
        s.remove_edges(torch.as_tensor(rem.view(np.int64), device=s.dev))
        new_uid = _u64(s.insert_edges(ns, nd, nL))
        keep = ~np.isin(live_uid, rem)
        live_uid = np.concatenate([live_uid[keep], new_uid])
        live_src = np.concatenate([live_src[keep], ns])
        live_dst = np.concatenate([live_dst[keep], nd])
        live_Lam = np.concatenate([live_Lam[keep], nL])
        cur = W.Model(model.q, model.lam, live_src, live_dst, live_Lam)
        assert sorted(_u64(s.live_uids()).tolist()) == sorted(live_uid.tolist())
        s.uids = torch.as_tensor(live_uid.view(np.int64), device=s.dev)
        dec = oracle.decompose(cur)
        x_in = _random_state(cur, C, 50 + rnd)
        r = teacher_forced(s, cur, dec, seed, x_in, 10 + rnd)
        _say(f"  round {rnd}: live={len(live_uid)} {r}")
        assert r["bad_dual"] == 0 and r["bad_x"] == 0, r
        s.sweep(2)
    # uids are never reused
    assert len(set(live_uid.tolist())) == len(live_uid)
    s.close()


def _new_edges(rng, model, k, focus=None, share=1.0):
    """k random edges (a share of them with src in `focus`), tables N(0, 0.5)
    zeroed beyond each endpoint's q."""
    n, qm = model.n, model.q_max
    src = rng.integers(0, n, size=k)
    if focus is not None:
        pick = rng.random(k) < share
        src[pick] = rng.choice(np.asarray(focus), size=int(pick.sum()))
    dst = (src + 1 + rng.integers(0, n - 1, size=k)) % n
    Lam = rng.normal(0.0, 0.5, size=(k, qm, qm))
    for e in range(k):
        Lam[e, model.q[src[e]]:, :] = 0.0
        Lam[e, :, model.q[dst[e]]:] = 0.0
    return src.astype(np.int32), dst.astype(np.int32), Lam.astype(model.Lam.dtype)


@pytest.mark.parametrize("C", [64, 8])
def test_store_growth_relocation_and_relayout(C):
    """Edit batches that grow one node into a hub, empty it and refill it,
    remove 40 % of the edges, and add more edges than the pool holds: segment
    relocation, full re-layout (fresh buffers), tombstone compaction and the
    hub table all run on the device.  After every batch the live uid set is
    checked and a teacher-forced sweep matches the oracle; a second context
    replaying the same batches issues the same uids and, after free sweeps,
    holds the same state bit for bit (the store's decisions are deterministic).
    64 chains: the 64-lane kernels; 8 chains: the 8-lane ones, hub pieces
    shared by eight lane groups."""
    import torch
    model = W.random_graph(600, 800, [2, 3, 4], seed=31, dtype="f32")
    seed = 9
    cap = 3400
    a = _sampler(model, C, seed, edge_capacity=cap)
    b = _sampler(model, C, seed, edge_capacity=cap)
    rng = np.random.default_rng(32)
    live_uid = _u64(a.uids).copy()
    assert np.array_equal(live_uid, _u64(b.uids))
    live = dict(src=model.src.copy(), dst=model.dst.copy(), Lam=model.Lam.copy())
    a.init()
    b.init()

    def insert(src, dst, Lam):
        nonlocal live_uid
        ua = _u64(a.insert_edges(src, dst, Lam))
        ub = _u64(b.insert_edges(src, dst, Lam))
        assert np.array_equal(ua, ub)
        live_uid = np.concatenate([live_uid, ua])
        for k, v in (("src", src), ("dst", dst), ("Lam", Lam)):
            live[k] = np.concatenate([live[k], v])

    def remove(mask):
        nonlocal live_uid
        rem = live_uid[mask]
        for s in (a, b):
            s.remove_edges(torch.as_tensor(rem.view(np.int64), device=s.dev))
        live_uid = live_uid[~mask]
        for k in live:
            live[k] = live[k][~mask]

    steps = [
        ("hub growth", lambda: insert(*_new_edges(rng, model, 600, focus=[0, 0, 0, 1, 2]))),
        ("remove 40%", lambda: remove(rng.random(len(live_uid)) < 0.4)),
        ("bulk insert", lambda: insert(*_new_edges(rng, model, 1500))),
        ("empty the hub", lambda: remove((live["src"] == 0) | (live["dst"] == 0))),
        ("refill the hub", lambda: insert(*_new_edges(rng, model, 300, focus=[0]))),
    ]
    for rnd, (name, step) in enumerate(steps):
        step()
        assert sorted(_u64(a.live_uids()).tolist()) == sorted(live_uid.tolist())
        cur = W.Model(model.q, model.lam, live["src"], live["dst"], live["Lam"])
        deg0 = int(np.count_nonzero(cur.src == 0) + np.count_nonzero(cur.dst == 0))
        a.uids = torch.as_tensor(live_uid.view(np.int64), device=a.dev)
        dec = oracle.decompose(cur)
        x_in = _random_state(cur, C, 70 + rnd)
        r = teacher_forced(a, cur, dec, seed, x_in, 20 + rnd)
        _say(f"  {name}: live={len(live_uid)} deg(0)={deg0} {r}")
        assert r["bad_dual"] == 0 and r["bad_x"] == 0, r
        assert r["flagged"] <= FLAG_BUDGET * r["draws"] + 2, r
        # the estimator reads the tables kept per slot: reused slots hold the new ones
        a.t = 30 + rnd
        a.set_state(torch.as_tensor(x_in, device=a.dev))
        a.dual_phase()
        lv = a.log_v().cpu().numpy()
        o = oracle.log_v(cur, dec, _u64(a.duals(a.uids)), x_in)
        assert (np.abs(lv - o) <= _log_v_tolerance(cur, x_in, o)).all(), (lv, o)
        a.primal_phase()
    x0 = _random_state(model, C, 99)
    for s in (a, b):
        s.set_state(torch.as_tensor(x0, device=s.dev))
        s.t = 40
        s.sweep(3)
    assert np.array_equal(a.state().cpu().numpy(), b.state().cpu().numpy())
    a.close()
    b.close()



def test_marginals_after_edits_vs_enumeration():
    """Statistical check through edits: a 3x3 q=3 grid (FP64, 64 chains) loses
    four edges and gains three new ones (two of them parallel to an existing
    edge); after burn-in the GPU marginals of the edited model agree with
    enumeration over its 19 683 states within 3.5 batch-means standard errors."""
    import torch
    from paper_1611_06684_amd import pdg
    model = W.table_grid(3, 3, 3, seed=61, pair_std=0.8, dtype="f64")
    C = 64
    s = _sampler(model, C, seed=8, burn_in=0, edge_capacity=model.m + 3)
    uids = _u64(s.uids)
    rng = np.random.default_rng(62)
    drop = np.sort(rng.choice(model.m, size=4, replace=False))
    s.remove_edges(uids[drop])
    ns, nd = np.array([0, 4, 8], np.int32), np.array([8, 5, 6], np.int32)
    nL = rng.normal(0.0, 0.8, size=(3, 3, 3))
    s.insert_edges(ns, nd, nL)
    keep = np.setdiff1d(np.arange(model.m), drop)
    cur = W.Model(model.q, model.lam, np.concatenate([model.src[keep], ns]),
                  np.concatenate([model.dst[keep], nd]), np.concatenate([model.Lam[keep], nL]))
    exact = brute.exact_marginals(cur)
    s.init()
    s.sweep(300)
    est = []
    cnt = torch.zeros((model.n, model.q_max), dtype=torch.int32, device=s.dev)
    for b in range(40):
        s.reset_marginals()
        s.sweep(100)
        n = pdg.pdg_get_counts(s.ctx, cnt.data_ptr())
        est.append(cnt.cpu().numpy() / n)
    mean, se = brute.batch_means(np.array(est))
    z = np.abs(mean - exact) / np.maximum(se, 1e-12)
    _say("  max z:", float(z.max()))
    assert (z < 3.5).all(), z
    s.close()

def test_checkpoint_resume_is_bit_exact():
    """A chain saved after t1 sweeps (state and sweep counter) and resumed in a
    fresh context continues exactly as the uninterrupted run: the generator is
    counter-based, so (x, t) is the whole state of a chain."""
    for model, C in [(W.table_grid(40, 30, 4, seed=21), 64), (W.chung_lu(2048, 5, seed=22), 32)]:
        seed, t1, t2 = 11, 3, 4
        a = _sampler(model, C, seed)
        a.init()
        a.sweep(t1 + t2)
        x_full = a.state().cpu().numpy()
        a.close()
        b = _sampler(model, C, seed)
        b.init()
        b.sweep(t1)
        x_mid, t_mid = b.state().clone(), b.t
        b.close()
        c = _sampler(model, C, seed)
        c.set_state(x_mid)
        c.t = t_mid
        c.sweep(t2)
        assert c.t == t1 + t2
        assert np.array_equal(c.state().cpu().numpy(), x_full)
        c.close()


def test_error_paths():
    import torch
    from paper_1611_06684_amd import pdg
    model = W.random_graph(50, 60, [3], seed=2, dtype="f32")
    s = _sampler(model, 4, 0, edge_capacity=62)
    dev = s.dev
    with pytest.raises(pdg.PdgError) as e:
        s.remove_edges(torch.tensor([12345], dtype=torch.int64, device=dev))
    assert e.value.code == pdg.PDG_ENOTFOUND
    u0 = s.uids[:1]
    with pytest.raises(pdg.PdgError) as e:  # repeated uid: nothing removed
        s.remove_edges(torch.cat([u0, u0]))
    assert e.value.code == pdg.PDG_ENOTFOUND
    assert pdg.pdg_num_edges(s.ctx) == 60
    with pytest.raises(pdg.PdgError) as e:
        s.insert_edges([1], [1], np.zeros((1, 3, 3), np.float32))
    assert e.value.code == pdg.PDG_EINVAL
    with pytest.raises(pdg.PdgError) as e:
        s.insert_edges([1], [99], np.zeros((1, 3, 3), np.float32))
    assert e.value.code == pdg.PDG_EINVAL
    bad = np.zeros((1, 3, 3), np.float32)
    bad[0, 1, 1] = np.nan
    with pytest.raises(pdg.PdgError) as e:
        s.insert_edges([1], [2], bad)
    assert e.value.code == pdg.PDG_ENONPOS
    with pytest.raises(pdg.PdgError) as e:
        s.insert_edges([1, 2, 3], [2, 3, 4], np.zeros((3, 3, 3), np.float32))
    assert e.value.code == pdg.PDG_ECAPACITY
    assert pdg.pdg_num_edges(s.ctx) == 60
    with pytest.raises(pdg.PdgError) as e:  # log V only between the phases
        s.log_v()
    assert e.value.code == pdg.PDG_ESTATE
    # a state out of range (x_i = q_i, in-bounds memory) is refused, nothing copied
    s.init()
    x_ok = s.state().clone()
    x_bad = x_ok.clone()
    x_bad[17, 2] = int(model.q[17])
    with pytest.raises(pdg.PdgError) as e:
        s.set_state(x_bad)
    assert e.value.code == pdg.PDG_EINVAL
    assert torch.equal(s.state(), x_ok)
    s.dual_phase()
    with pytest.raises(pdg.PdgError) as e:
        s.insert_edges([1], [2], np.zeros((1, 3, 3), np.float32))
    assert e.value.code == pdg.PDG_ESTATE
    with pytest.raises(pdg.PdgError) as e:
        s.dual_phase()
    assert e.value.code == pdg.PDG_ESTATE
    s.primal_phase()
    s.sync()
    s.close()


def test_full_size_plain_grid_sampled():
    """Plain grid workload at full size (1024x1024, q=4, FP32 tables, 64 chains),
    in the launch configuration the benchmark times: one sweep from init, then
    sampled nodes and their incident edges checked one by one by the oracle."""
    import torch
    model = W.table_grid(1024, 1024, 4, seed=0)
    C, seed = 64, 0
    _say(f"[full-size] n={model.n} m={model.m}")
    s = _sampler(model, C, seed)
    s.init()
    s.sweep(3)
    x_prev = s.state().cpu().numpy()
    s.dual_phase()
    # Sec. 5.2 estimator at full size: log V of two chains against the oracle
    lv = s.log_v().cpu().numpy()
    th2 = np.ascontiguousarray(_u64(s.duals(s.uids))[:, :2])
    dec_full = oracle.decompose(model)
    o = oracle.log_v(model, dec_full, th2, np.ascontiguousarray(x_prev[:, :2]))
    tol = _log_v_tolerance(model, np.ascontiguousarray(x_prev[:, :2]), o)
    _say(f"[full-size] log V {lv[:2]} vs oracle {o}, tol {tol}")
    assert (np.abs(lv[:2] - o) <= tol).all()
    del th2, dec_full
    uids = _u64(s.uids)
    rng = np.random.default_rng(0)
    nodes = rng.choice(model.n, size=300, replace=False)
    # incident edges of the sampled nodes (grid: src/dst lookup)
    order = np.argsort(np.concatenate([model.src, model.dst]), kind="stable")
    ends = np.concatenate([model.src, model.dst])[order]
    lo, hi = np.searchsorted(ends, nodes), np.searchsorted(ends, nodes, side="right")
    inc = {int(i): order[a:b] for i, a, b in zip(nodes, lo, hi)}
    edges = np.unique(np.concatenate(list(inc.values())) % model.m)
    th_g = _u64(s.duals(torch.as_tensor(uids[edges].view(np.int64), device=s.dev)))
    s.primal_phase()
    x_new = s.state().cpu().numpy()
    t = s.t
    subm = model.subset_edges(edges)
    dec = oracle.decompose(subm)
    sub = {int(e): k for k, e in enumerate(edges)}
    n_draw = n_flag = 0
    for k, e in enumerate(edges):
        for c in range(C):
            th, fl = oracle.dual_edge(subm, dec, k,
                                      x_prev[model.src[e], c], x_prev[model.dst[e], c],
                                      uids[e], c, t, seed)
            assert ((int(th_g[k, c]) ^ th) & ~fl) == 0, (e, c)
            n_draw += 9
            n_flag += bin(fl).count("1")
    for i in nodes:
        es = inc[int(i)]
        sides = (es >= model.m).astype(np.int32)
        rows = np.array([sub[int(e % model.m)] for e in es])
        for c in range(C):
            xo, fo = oracle.primal_node(subm, dec, int(i), rows, sides,
                                        [th_g[r, c] for r in rows], c, t, seed)
            assert fo or xo == x_new[i, c], (i, c)
            n_draw += 1
            n_flag += fo
    _say(f"  sampled draws {n_draw}, flagged {n_flag}")
    assert n_flag <= max(FLAG_BUDGET * n_draw, 3)
    s.close()


def test_full_size_dynamic_sparse_sampled():
    """Dynamic sparse workload at full size (Chung-Lu, 2^22 nodes, q=8, FP32
    tables, 32 chains) in the launch configuration the benchmark times: sweeps
    from init, one 1 % churn batch, a sweep on the edited graph, then one sweep
    whose sampled edges and nodes -- the three largest hubs among them -- are
    checked one by one by the oracle."""
    import torch
    n, q, C, seed = 1 << 22, 8, 32, 0
    _say("[dynamic full-size] building the graph")
    model = W.chung_lu(n, q, seed=0)
    _say(f"[dynamic full-size] n={model.n} m={model.m}; uploading")
    s = _sampler(model, C, seed, edge_capacity=model.m)
    s.init()
    s.sweep(2)
    live_uid = _u64(s.uids).copy()
    live_src, live_dst = model.src.copy(), model.dst.copy()
    live_tab = np.arange(model.m)               # row of Lam for each live edge
    churn = W.Churn(n, q, model.meta["weights"], seed=1)
    rem, ns, nd, nL = churn.next_batch(live_uid)
    _say(f"[dynamic full-size] churn: {len(rem)} removals and insertions")
    s.remove_edges(torch.as_tensor(rem.view(np.int64), device=s.dev))
    new_uid = _u64(s.insert_edges(ns, nd, nL))
    keep = ~np.isin(live_uid, rem)
    live_uid = np.concatenate([live_uid[keep], new_uid])
    live_src = np.concatenate([live_src[keep], ns])
    live_dst = np.concatenate([live_dst[keep], nd])
    live_tab = np.concatenate([live_tab[keep], model.m + np.arange(len(ns))])
    Lam_all = np.concatenate([model.Lam, nL])
    s.sweep(1)
    x_prev = s.state().cpu().numpy()
    s.dual_phase()
    deg = np.bincount(np.concatenate([live_src, live_dst]), minlength=n)
    hubs = np.argsort(deg)[-3:]
    rng = np.random.default_rng(0)
    nodes = np.unique(np.concatenate([rng.choice(n, size=150, replace=False), hubs]))
    ends = np.concatenate([live_src, live_dst])
    order = np.argsort(ends, kind="stable")
    se = ends[order]
    lo, hi = np.searchsorted(se, nodes), np.searchsorted(se, nodes, side="right")
    m_live = len(live_uid)
    inc = {int(i): order[a:b] for i, a, b in zip(nodes, lo, hi)}
    edges = np.unique(np.concatenate([v % m_live for v in inc.values()]))
    _say(f"[dynamic full-size] {len(nodes)} nodes (max degree {deg.max()}), {len(edges)} edges")
    th_g = _u64(s.duals(torch.as_tensor(live_uid[edges].view(np.int64), device=s.dev)))
    s.primal_phase()
    x_new = s.state().cpu().numpy()
    t = s.t
    subm = W.Model(model.q, model.lam, live_src[edges], live_dst[edges], Lam_all[live_tab[edges]])
    dec = oracle.decompose(subm)
    sub = {int(e): k for k, e in enumerate(edges)}
    n_draw = n_flag = 0
    for k, e in enumerate(edges):
        for c in range(C):
            th, fl = oracle.dual_edge(subm, dec, k, x_prev[live_src[e], c], x_prev[live_dst[e], c],
                                      live_uid[e], c, t, seed)
            assert ((int(th_g[k, c]) ^ th) & ~fl) == 0, (e, c)
            n_draw += 49
            n_flag += bin(fl).count("1")
    for i in nodes:
        es = inc[int(i)]
        sides = (es >= m_live).astype(np.int32)
        rows = np.array([sub[int(e % m_live)] for e in es], dtype=np.int64)
        for c in range(C):
            xo, fo = oracle.primal_node(subm, dec, int(i), rows, sides,
                                        [th_g[r, c] for r in rows], c, t, seed)
            assert fo or xo == x_new[i, c], (i, c)
            n_draw += 1
            n_flag += fo
    _say(f"  sampled draws {n_draw}, flagged {n_flag}")
    assert n_flag <= max(FLAG_BUDGET * n_draw, 3)
    s.close()


def test_full_size_batched_by_states_sampled():
    """Batched workload at its full recipe (4096 graphs: sparse with q in
    {2,3,5}, 64 dense binary graphs on 2048 nodes; FP32 tables; 8 chains) in
    the configuration the benchmark times: one context per state count, each
    tuned by pdg_tune, sweeps replayed from one captured HIP graph.  After two
    replays, the draws of a third are checked on sampled nodes (two of them in
    dense graphs, 2047 incidences each) and all their incident edges, one by
    one, against the oracle."""
    import torch
    from paper_1611_06684_amd import pdg
    C = 8
    _say("[batched full-size] building the batch per state count")
    groups = W.batched_by_states(4096, 64, seed=0)
    samplers = []
    for k, (q, model) in enumerate(groups):
        _say(f"[batched full-size] q={q}: n={model.n} m={model.m}, seed {k}")
        s = _sampler(model, C, k)
        s.init()
        tun = pdg.pdg_tune(s.ctx, 2)
        _say(f"  tuning {tun.as_dict()}")
        samplers.append(s)
    graph = pdg.pdg_graph_create([s.ctx for s in samplers], 1)
    pdg.pdg_graph_launch(graph)
    pdg.pdg_graph_launch(graph)
    x_prev = [s.state().cpu().numpy() for s in samplers]
    pdg.pdg_graph_launch(graph)
    pdg.pdg_graph_destroy(graph)
    rng = np.random.default_rng(0)
    for k, ((q, model), s) in enumerate(zip(groups, samplers)):
        seed = k
        t = s.t
        assert t == 3
        uids = _u64(s.uids)
        nodes = rng.choice(model.n, size=60, replace=False)
        if q == 2:  # the dense graphs come first in the binary context
            nodes = np.unique(np.concatenate([nodes, [5, 2048 * 63 + 100]]))
        ends = np.concatenate([model.src, model.dst])
        order = np.argsort(ends, kind="stable")
        se = ends[order]
        lo, hi = np.searchsorted(se, nodes), np.searchsorted(se, nodes, side="right")
        inc = {int(i): order[a:b] for i, a, b in zip(nodes, lo, hi)}
        edges = np.unique(np.concatenate(list(inc.values())) % model.m)
        th_g = _u64(s.duals(torch.as_tensor(uids[edges].view(np.int64), device=s.dev)))
        x_new = s.state().cpu().numpy()
        subm = model.subset_edges(edges)
        dec = oracle.decompose(subm)
        sub = {int(e): j for j, e in enumerate(edges)}
        n_draw = n_flag = 0
        xp = x_prev[k]
        for j, e in enumerate(edges):
            for c in range(C):
                th, fl = oracle.dual_edge(subm, dec, j, xp[model.src[e], c], xp[model.dst[e], c],
                                          uids[e], c, t, seed)
                assert ((int(th_g[j, c]) ^ th) & ~fl) == 0, (q, e, c)
                n_draw += (q - 1) * (q - 1)
                n_flag += bin(fl).count("1")
        for i in nodes:
            es = inc[int(i)]
            sides = (es >= model.m).astype(np.int32)
            rows = np.array([sub[int(e % model.m)] for e in es], dtype=np.int64)
            for c in range(C):
                xo, fo = oracle.primal_node(subm, dec, int(i), rows, sides,
                                            [th_g[r, c] for r in rows], c, t, seed)
                assert fo or xo == x_new[i, c], (q, i, c)
                n_draw += 1
                n_flag += fo
        _say(f"  q={q}: {len(nodes)} nodes, {len(edges)} edges, sampled draws {n_draw}, "
             f"flagged {n_flag}")
        assert n_flag <= max(FLAG_BUDGET * n_draw, 3)
    for s in samplers:
        s.close()
