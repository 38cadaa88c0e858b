"""Brute-force references for tiny models (plain definitions, numpy FP64).

* ``log_joint`` / ``exact_marginals``: the MRF itself,
  p(x) proportional to prod_i u_i(x_i) prod_e phi_e(x_src, x_dst) (the target
  the sampler must leave invariant, paper Sec. 3 / Sec. 5.1), by enumeration.
* ``exact_transition``: the exact one-sweep transition matrix of the x-chain,
  T(x -> x') = sum_theta p(theta | x) p(x' | theta), enumerating every dual
  configuration and taking the two conditionals from the oracle's probability
  functions (not from its sampler).
* ``joint``: the primal-dual joint p(x, theta) = p(x) p(theta | x) over every
  state and dual configuration (the x-marginal is the MRF by construction;
  p(theta | x) from the oracle's dual probability function).
* ``batch_means``: Monte-Carlo standard errors of marginal estimates.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle


def all_states(q) -> np.ndarray:
    grids = np.meshgrid(*[np.arange(int(qi)) for qi in q], indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1)


def log_joint(model, X) -> np.ndarray:
    lam = np.asarray(model.lam, np.float64)
    Lam = np.asarray(model.Lam, np.float64)
    lp = np.zeros(X.shape[0])
    for i in range(model.n):
        lp += lam[i, X[:, i]]
    for e in range(model.m):
        lp += Lam[e, X[:, model.src[e]], X[:, model.dst[e]]]
    return lp


def stationary(model):
    X = all_states(model.q)
    lp = log_joint(model, X)
    p = np.exp(lp - lp.max())
    return X, p / p.sum()


def exact_marginals(model) -> np.ndarray:
    X, p = stationary(model)
    out = np.zeros((model.n, model.q_max))
    for i in range(model.n):
        for a in range(int(model.q[i])):
            out[i, a] = p[X[:, i] == a].sum()
    return out


def _softmax_rows(L, q):
    out = np.zeros_like(L)
    for i in range(L.shape[0]):
        v = L[i, : q[i]]
        w = np.exp(v - v.max())
        out[i, : q[i]] = w / w.sum()
    return out


def _dual_bits(model):
    bits = []  # (edge, d, a, b)
    for e in range(model.m):
        qi, qj = int(model.q[model.src[e]]), int(model.q[model.dst[e]])
        for a in range(1, qi):
            for b in range(1, qj):
                bits.append((e, (a - 1) * (qj - 1) + (b - 1), a, b))
    assert len(bits) <= 14, "too many duals to enumerate"
    return bits


def _dual_probabilities(model, dec, X, bits):
    """p(theta | x) [S][K] for every dual configuration k (bit k of the
    enumeration = bits[k]), and the configurations as theta arrays [K][m]."""
    S, nb = X.shape[0], len(bits)
    K = 1 << nb
    p1 = np.zeros((S, nb))
    for k, (e, d, a, b) in enumerate(bits):
        ys = (X[:, model.src[e]] == a).astype(int)
        yd = (X[:, model.dst[e]] == b).astype(int)
        tab = {(y, yp): oracle.dual_p1(dec.par[e, d], y, yp) for y in (0, 1) for yp in (0, 1)}
        p1[:, k] = [tab[(int(u), int(v))] for u, v in zip(ys, yd)]
    cfg = ((np.arange(K)[:, None] >> np.arange(nb)[None, :]) & 1).astype(np.float64)
    P_th = np.exp(np.log(p1) @ cfg.T + np.log1p(-p1) @ (1.0 - cfg).T)  # [S][K]
    TH = np.zeros((K, model.m), np.uint64)
    for kk in range(K):
        for k, (e, d, a, b) in enumerate(bits):
            if (kk >> k) & 1:
                TH[kk, e] |= np.uint64(1) << np.uint64(d)
    return P_th, TH


def exact_transition(model, dec):
    """Returns (X, T) with T[s, s'] = P(x_{t} = X[s'] | x_{t-1} = X[s])."""
    X = all_states(model.q)
    S = X.shape[0]
    bits = _dual_bits(model)
    P_th, TH = _dual_probabilities(model, dec, X, bits)
    K = P_th.shape[1]
    # p(x' | theta): product over nodes of the categorical conditionals
    P_x = np.zeros((K, S))
    for kk in range(K):
        L = oracle.all_logits(model, dec, TH[kk])
        pr = _softmax_rows(L, model.q)
        P_x[kk] = np.prod(pr[np.arange(model.n)[None, :], X], axis=1)
    return X, P_th @ P_x


def joint(model, dec):
    """Returns (X [S][n], TH [K][m] u64, P [S][K]) with P[s, k] = p(X[s], TH[k])."""
    X, px = stationary(model)
    bits = _dual_bits(model)
    P_th, TH = _dual_probabilities(model, dec, X, bits)
    return X, TH, px[:, None] * P_th


def batch_means(series_counts: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """series_counts: [n_batches][...] per-batch frequency estimates (equal batch
    sizes).  Returns (mean, standard error of the mean)."""
    nb = series_counts.shape[0]
    mean = series_counts.mean(axis=0)
    se = series_counts.std(axis=0, ddof=1) / np.sqrt(nb)
    return mean, se
