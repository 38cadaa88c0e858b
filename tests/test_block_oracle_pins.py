"""Pins of the learned-block-proposal oracle (blocking of Sec. 5.4) against
facts that do not come from it: the block conditional against brute force over
the MRF and the dual conditional; Metropolis-Hastings detailed balance and
stationarity by enumeration; acceptance 1 for an exact proposal; sampled
transition frequencies; a whole learned step leaving p(x) invariant on a tiny
grid; network gradients against finite differences; Adam's first step in
closed form."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import block_oracle as B
from oracle import oracle
from paper_1611_06684_amd import workloads as W


def _grid(H, Wd, seed, J=(0.0, 0.6), hstd=0.4):
    rng = np.random.default_rng(seed)
    src, dst = W.grid_edges(H, Wd)
    Jv = rng.uniform(J[0], J[1], size=src.shape[0])
    h = rng.normal(0, hstd, size=H * Wd)
    return W.ising_model(src, dst, Jv, h, H * Wd)


def _table_grid(H, Wd, seed):
    """Binary grid with general (not symmetric) 2x2 log-tables N(0, 0.5)."""
    return W.table_grid(H, Wd, 2, seed=seed, pair_std=0.5, unary_std=0.5, dtype="f64")


def _log_joint(model, X):
    """log p~(x) of the MRF definition for rows X [k][n] of 0/1 states."""
    lam, Lam = np.asarray(model.lam, float), np.asarray(model.Lam, float)
    out = lam[np.arange(model.n), X].sum(-1)
    out += Lam[np.arange(model.m), X[:, model.src], X[:, model.dst]].sum(-1)
    return out


def _all_states(k):
    return np.array(list(itertools.product([0, 1], repeat=k)), np.int64)


def test_block_conditional_is_the_mrf_given_cut_duals():
    """p(x_B | theta_cut, x_rest) from brute force over p(x) prod_cut p(theta_e|x)
    (the dual conditional of the decomposition) equals the oracle's
    exp(f x + x^T K x) normalised, for every block, cut-dual configuration and
    two settings of the rest of the grid (the conditional must not depend on it)."""
    model = _table_grid(4, 4, 1)  # general tables: both odds-ratio signs, asymmetric rows/columns
    blk = B.Blocking(4, 4, 2)
    dec = oracle.decompose(model)
    cut = np.flatnonzero(blk.cut)
    lor = model.Lam[:, 1, 1] + model.Lam[:, 0, 0] - model.Lam[:, 1, 0] - model.Lam[:, 0, 1]
    assert (lor[cut] < 0).any() and (lor[cut] > 0).any()
    rng = np.random.default_rng(2)
    for trial in range(6):
        th_cut = rng.integers(0, 2, size=len(cut))
        theta = np.zeros((model.m, 1), np.uint8)
        theta[cut, 0] = th_cut
        f, internal = B.block_fields(model, dec, blk, theta)
        K = B.block_couplings(blk, internal)
        for b in range(blk.nb):
            nodes = blk.nodes[b]
            XB = _all_states(4)
            want = B.log_ptilde(XB, f[b, 0], K[b])
            want = np.exp(want - want.max())
            want /= want.sum()
            for rest_seed in (3, 4):
                x_rest = np.random.default_rng(rest_seed + trial).integers(0, 2, size=model.n)
                X = np.repeat(x_rest[None, :], 16, axis=0)
                X[:, nodes] = XB
                lp = _log_joint(model, X)
                for k, e in enumerate(cut):
                    p1 = np.array([oracle.dual_p1(dec.par[e, 0], X[r, model.src[e]],
                                                  X[r, model.dst[e]]) for r in range(16)])
                    lp += np.log(p1 if th_cut[k] else 1.0 - p1)
                got = np.exp(lp - lp.max())
                got /= got.sum()
                np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)


def _mh_matrix(f, K, logits):
    k = len(f)
    S = _all_states(k)
    lq = B.proposal_logprob(S, logits)
    T = np.zeros((len(S), len(S)))
    for a in range(len(S)):
        la = B.mh_log_accept(np.repeat(S[a][None], len(S), 0), S, f, K, logits)
        T[a] = np.exp(lq) * np.minimum(1.0, np.exp(la))
        T[a, a] = 0.0
        T[a, a] = 1.0 - T[a].sum()
    return S, T


@pytest.mark.parametrize("bs,seed", [(2, 5), (3, 6)])
def test_mh_kernel_detailed_balance_and_stationarity(bs, seed):
    """The MH transition matrix of one block (2x2: 16 states; 3x3: 512), built
    from the proposal probabilities and the acceptance of the oracle with
    arbitrary logits, satisfies detailed balance and pi T = pi for pi the block
    conditional exp(f x + x^T K x) normalised."""
    rng = np.random.default_rng(seed)
    k = bs * bs
    blk = B.Blocking(bs, bs, bs)
    model = _grid(bs, bs, seed, J=(-0.5, 0.8))
    dec = oracle.decompose(model)
    f, internal = B.block_fields(model, dec, blk, np.zeros((model.m, 1), np.uint8))
    K = B.block_couplings(blk, internal)[0]
    f = f[0, 0] + rng.normal(0, 0.5, size=k)
    logits = rng.normal(0, 1.0, size=k)
    S, T = _mh_matrix(f, K, logits)
    lp = B.log_ptilde(S, f, K)
    pi = np.exp(lp - lp.max())
    pi /= pi.sum()
    F = pi[:, None] * T
    np.testing.assert_allclose(F, F.T, atol=1e-15)
    np.testing.assert_allclose(pi @ T, pi, atol=1e-14)
    assert (T >= -1e-15).all()


def test_exact_proposal_is_always_accepted():
    """Without internal couplings the block conditional is the product of
    Bernoulli(sigmoid(f_i)); with logits = f every proposal is accepted."""
    rng = np.random.default_rng(7)
    k = 9
    f = rng.normal(0, 1, size=k)
    K = np.zeros((k, k))
    S = _all_states(k)
    for a in rng.choice(len(S), size=20, replace=False):
        la = B.mh_log_accept(np.repeat(S[a][None], len(S), 0), S, f, K, f)
        np.testing.assert_allclose(la, 0.0, atol=1e-13)
    # and through the sampler: a 3x3 grid cut into 3x3 blocks whose only edges
    # are zero-coupling ones
    model = W.ising_model(*W.grid_edges(3, 3), np.zeros(12), rng.normal(0, 1, 9), 9)
    blk = B.Blocking(3, 3, 3)
    dec = oracle.decompose(model)
    x = rng.integers(0, 2, size=(9, 16)).astype(np.uint8)
    th, _ = B.cut_duals(model, dec, blk, x, 3, 1)
    fb, internal = B.block_fields(model, dec, blk, th)
    Kb = B.block_couplings(blk, internal)
    _, acc, _, _ = B.mh_step(blk, x, fb, Kb, fb.copy(), 3, 1)
    assert acc.all()


def test_sampled_transitions_match_the_mh_matrix():
    """Empirical transitions of the oracle's Philox-driven proposal and
    acceptance from one 2x2 state, over 40 000 steps, against the enumerated
    MH row (chi-square, 15 dof, p ~ 1e-6 threshold)."""
    rng = np.random.default_rng(8)
    model = _grid(2, 2, 9, J=(0.2, 0.9))
    blk = B.Blocking(2, 2, 2)
    dec = oracle.decompose(model)
    f, internal = B.block_fields(model, dec, blk, np.zeros((model.m, 1), np.uint8))
    K = B.block_couplings(blk, internal)
    logits = rng.normal(0, 1, size=4)
    S, T = _mh_matrix(f[0, 0], K[0], logits)
    x0 = np.array([1, 0, 0, 1], np.uint8)
    a = int(np.flatnonzero((S == x0).all(1))[0])
    C, steps = 400, 100
    x = np.repeat(x0[:, None], C, axis=1)
    counts = np.zeros(16)
    fC = np.repeat(f, C, axis=1)
    lC = np.broadcast_to(logits, (1, C, 4)).astype(np.float32).astype(np.float64)
    for s in range(1, steps + 1):
        xn, _, _, _ = B.mh_step(blk, x, fC, K, lC, 11, s)
        idx = (xn.T[:, None, :] == S[None]).all(-1).argmax(-1)
        counts += np.bincount(idx, minlength=16)
    _, T32 = _mh_matrix(f[0, 0], K[0], lC[0, 0])
    exp = T32[a] * C * steps
    keep = exp > 5
    chi2 = ((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert chi2 < 50, (chi2, counts, exp)
    assert counts[~keep].sum() < 40


def test_learned_step_leaves_the_joint_invariant():
    """A whole learned step on a 2x4 grid cut into two 2x2 blocks -- cut duals
    from x, fields, logits from a small random network of the duals and
    fields, MH per block -- has a transition matrix (enumerated over the 4
    cut-dual configurations and all proposals) with pi T = pi, pi the MRF."""
    model = _table_grid(2, 4, 12)
    blk = B.Blocking(2, 4, 2)
    dec = oracle.decompose(model)
    rng = np.random.default_rng(13)
    nin, k = 4 + 8, 4
    P = {"W1": B.bf16(rng.normal(0, 0.5, (6, nin))), "b1": rng.normal(0, 0.1, 6),
         "W2": B.bf16(rng.normal(0, 0.5, (6, 6))), "b2": rng.normal(0, 0.1, 6),
         "W3": B.bf16(rng.normal(0, 0.5, (k, 6))), "b3": rng.normal(0, 0.1, k)}
    S = _all_states(8)
    cut = np.flatnonzero(blk.cut)
    Tfull = np.zeros((256, 256))
    for a, xs in enumerate(S):
        for tc in itertools.product([0, 1], repeat=len(cut)):
            pt = 1.0
            for e, t in zip(cut, tc):
                p1 = oracle.dual_p1(dec.par[e, 0], xs[model.src[e]], xs[model.dst[e]])
                pt *= p1 if t else 1 - p1
            theta = np.zeros((model.m, 1), np.uint8)
            theta[cut, 0] = tc
            f, internal = B.block_fields(model, dec, blk, theta)
            K = B.block_couplings(blk, internal)
            _, _, L = B.mlp_forward(P, B.mlp_inputs(blk, f, theta))
            rows = []
            for b in range(2):
                Sb, Tb = _mh_matrix(f[b, 0], K[b], L[b])
                xb = xs[blk.nodes[b]]
                rows.append(Tb[int(np.flatnonzero((Sb == xb).all(1))[0])])
            for c, xt in enumerate(S):
                i0 = int(xt[blk.nodes[0]] @ (1 << np.arange(3, -1, -1)))
                i1 = int(xt[blk.nodes[1]] @ (1 << np.arange(3, -1, -1)))
                Tfull[a, c] += pt * rows[0][i0] * rows[1][i1]
    lp = _log_joint(model, S)
    pi = np.exp(lp - lp.max())
    pi /= pi.sum()
    np.testing.assert_allclose(Tfull.sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(pi @ Tfull, pi, atol=1e-13)


def test_mlp_gradients_match_finite_differences():
    """Backward pass of the network (without BF16 rounding) against central
    differences of the loss, for every weight and bias matrix."""
    rng = np.random.default_rng(14)
    nin, h, k, R = 10, 7, 4, 6
    P = {"W1": rng.normal(0, 0.4, (h, nin)), "b1": rng.normal(0, 0.3, h),
         "W2": rng.normal(0, 0.4, (h, h)), "b2": rng.normal(0, 0.3, h),
         "W3": rng.normal(0, 0.4, (k, h)), "b3": rng.normal(0, 0.3, k)}
    X = rng.normal(0, 1, (R, nin))
    T = rng.integers(0, 2, (R, k)).astype(float)
    H1, H2, L = B.mlp_forward(P, X, rounding=False)
    g = B.mlp_backward(P, X, H1, H2, L, T, rounding=False)
    eps = 1e-6
    for name in P:
        num = np.zeros_like(P[name])
        it = np.nditer(P[name], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            Pp = {kk: v.copy() for kk, v in P.items()}
            Pm = {kk: v.copy() for kk, v in P.items()}
            Pp[name][idx] += eps
            Pm[name][idx] -= eps
            num[idx] = (B.mlp_loss(B.mlp_forward(Pp, X, False)[2], T) -
                        B.mlp_loss(B.mlp_forward(Pm, X, False)[2], T)) / (2 * eps)
        np.testing.assert_allclose(g[name], num, rtol=1e-5, atol=1e-8, err_msg=name)


def test_adam_first_step_closed_form():
    """From m = v = 0 the bias-corrected first step is -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-9, 0.0])
    w = np.array([1.0, 1.0, 1.0, 1.0])
    w1, m, v = B.adam(w, g, np.zeros(4), np.zeros(4), 1, 0.01)
    np.testing.assert_allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_rounding_is_nearest_even():
    """bf16 keeps 8 significant bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7
    and goes to the even 1; 1 + 3 * 2^-8 goes up to 1 + 2^-6; values already
    representable are unchanged."""
    v = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 0.0, 1 + 2 ** -9])
    np.testing.assert_array_equal(B.bf16(v), [1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5, 0.0, 1.0])


def test_cut_dual_frequencies_match_the_dual_conditional():
    """Cut duals drawn by the oracle over 3000 steps from a fixed state: the
    frequency of theta_e = 1 on every cut edge and chain matches p(theta = 1 |
    x) of the decomposition within 5 binomial standard errors."""
    model = _grid(4, 4, 15, J=(-0.8, 0.8))
    blk = B.Blocking(4, 4, 2)
    dec = oracle.decompose(model)
    rng = np.random.default_rng(16)
    C = 4
    x = rng.integers(0, 2, size=(model.n, C)).astype(np.uint8)
    cut = np.flatnonzero(blk.cut)
    acc = np.zeros((model.m, C))
    steps = 3000
    for s in range(1, steps + 1):
        th, _ = B.cut_duals(model, dec, blk, x, 21, s)
        acc += th
    for e in cut:
        for c in range(C):
            p = oracle.dual_p1(dec.par[e, 0], x[model.src[e], c], x[model.dst[e], c])
            se = np.sqrt(p * (1 - p) / steps)
            assert abs(acc[e, c] / steps - p) < 5 * se + 1e-12, (e, c, acc[e, c] / steps, p)
    assert not acc[~blk.cut].any()
