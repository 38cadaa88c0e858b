"""Convergence and efficiency diagnostics of sampler output (host side, numpy).

These measure chains; they are not part of the sweep.  The paper judges mixing
by the potential scale reduction factor over parallel chains and a mixing time
read off it (Sec. 6); effective sample size is the usual companion measure.

* ``psrf_binary``: Gelman-Rubin R-hat of per-node indicator series from the
  chains' window means (for a 0/1 series the within-chain sample variance is
  p(1 - p) L / (L - 1), so means are all it needs).
* ``psrf``: the same from raw series (any scalar).
* ``mixing_time``: first evaluation point after which the PSRF stays below a
  threshold (Sec. 6: the first index so that the PSRF remains below it).
* ``ess``: effective sample size of pooled chains by Geyer's initial monotone
  sequence over the multi-chain autocorrelation (within-chain autocovariances
  averaged, combined with the between-chain variance).
"""
from __future__ import annotations

import numpy as np


def psrf_binary(means: np.ndarray, L: int) -> np.ndarray:
    """R-hat per series from window means of 0/1 data.

    means: [M chains, ...] fraction of ones of each chain over its window of L
    samples.  W = mean over chains of p(1-p) L/(L-1); B/L = variance of the
    chain means (ddof 1); var+ = (L-1)/L W + B/L; R-hat = sqrt(var+ / W).
    Series with W = 0 (every chain constant) give 1 when the chains agree and
    inf when they do not."""
    p = np.asarray(means, np.float64)
    M = p.shape[0]
    W = (p * (1.0 - p)).mean(axis=0) * L / (L - 1.0)
    B_over_L = p.var(axis=0, ddof=1) if M > 1 else np.zeros(p.shape[1:])
    var_plus = (L - 1.0) / L * W + B_over_L
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.sqrt(var_plus / W)
    r = np.where(W > 0, r, np.where(B_over_L > 0, np.inf, 1.0))
    return r


def psrf(series: np.ndarray) -> np.ndarray:
    """R-hat from raw series [M chains, L samples, ...]."""
    x = np.asarray(series, np.float64)
    M, L = x.shape[0], x.shape[1]
    W = x.var(axis=1, ddof=1).mean(axis=0)
    B_over_L = x.mean(axis=1).var(axis=0, ddof=1)
    var_plus = (L - 1.0) / L * W + B_over_L
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.sqrt(var_plus / W)
    return np.where(W > 0, r, np.where(B_over_L > 0, np.inf, 1.0))


def mixing_time(times, values, threshold: float = 1.01):
    """First time t_k such that values[j] < threshold for every j >= k; None when
    the last value is not below the threshold."""
    v = np.asarray(values)
    above = np.flatnonzero(~(v < threshold))
    if above.size == 0:
        return times[0]
    k = above[-1] + 1
    return times[k] if k < len(times) else None


def _autocov_fft(x: np.ndarray) -> np.ndarray:
    """Biased autocovariance of each row of x [M, L] at lags 0..L-1."""
    M, L = x.shape
    xc = x - x.mean(axis=1, keepdims=True)
    n = 1 << int(np.ceil(np.log2(2 * L)))
    f = np.fft.rfft(xc, n=n, axis=1)
    ac = np.fft.irfft(f * np.conj(f), n=n, axis=1)[:, :L]
    return ac / L


def ess(series: np.ndarray) -> float:
    """Effective sample size of M chains x L samples of one scalar, pooled.

    rho_t = 1 - (W - mean_m acov_m(t)) / var+, with W the mean within-chain
    variance (ddof 1) and var+ = (L-1)/L W + B/L.  Geyer's initial positive
    sequence: P_k = rho_2k + rho_2k+1 summed while positive, made monotone
    non-increasing; ESS = M L / (-1 + 2 sum_k P_k).  A constant series has ESS
    M L when the chains agree (no variance to estimate)."""
    x = np.asarray(series, np.float64)
    M, L = x.shape
    if L < 4:
        return float(M * L)
    acov = _autocov_fft(x)
    W = acov[:, 0].mean() * L / (L - 1.0)
    B_over_L = x.mean(axis=1).var(ddof=1) if M > 1 else 0.0
    var_plus = (L - 1.0) / L * W + B_over_L
    if var_plus <= 0:
        return float(M * L)
    rho = 1.0 - (W - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    npair = L // 2
    P = rho[0:2 * npair:2] + rho[1:2 * npair:2]
    # initial positive sequence, then monotone
    k_end = npair
    for k in range(npair):
        if P[k] <= 0:
            k_end = k
            break
    P = P[:k_end]
    if P.size == 0:
        return float(M * L)
    P = np.minimum.accumulate(P)
    tau = -1.0 + 2.0 * P.sum()
    return float(M * L / max(tau, 1e-12))
