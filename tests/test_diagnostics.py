"""Pins of the chain diagnostics against closed forms (CPU)."""
from __future__ import annotations

import numpy as np

from paper_1611_06684_amd import diagnostics as dg


def _ar1(rng, M, L, phi):
    """M stationary AR(1) chains x_t = phi x_{t-1} + e_t, unit innovations."""
    x = np.zeros((M, L))
    x[:, 0] = rng.normal(0, 1 / np.sqrt(1 - phi * phi), size=M)
    e = rng.normal(size=(M, L))
    for t in range(1, L):
        x[:, t] = phi * x[:, t - 1] + e[:, t]
    return x


def test_ess_of_ar1_matches_closed_form():
    """For AR(1) with coefficient phi the integrated autocorrelation time is
    (1 + phi) / (1 - phi), so ESS = M L (1 - phi) / (1 + phi)."""
    rng = np.random.default_rng(0)
    M, L = 8, 20000
    for phi in (0.0, 0.5, 0.9, -0.4):
        x = _ar1(rng, M, L, phi)
        want = M * L * (1 - phi) / (1 + phi)
        got = dg.ess(x)
        assert abs(got / want - 1) < 0.12, (phi, got, want)


def test_ess_counts_stuck_chains_as_few_samples():
    """Chains stuck at different values: the between-chain variance dominates and
    the ESS collapses towards the number of chains."""
    rng = np.random.default_rng(1)
    M, L = 6, 4000
    x = rng.normal(size=(M, L)) * 0.01 + np.arange(M)[:, None]
    assert dg.ess(x) < 0.05 * M * L


def test_psrf_closed_form_and_limits():
    """Two chains of L = 4 with means 0.25 and 0.75: W = (3/16 * 4/3) = 1/4,
    B/L = var([.25, .75], ddof 1) = 1/8, var+ = 3/4 * 1/4 + 1/8 = 5/16,
    R-hat = sqrt(5/4).  Raw series agree with the binary form; iid chains give
    R-hat near 1; chains that never move give inf when they disagree."""
    r = dg.psrf_binary(np.array([[0.25], [0.75]]), 4)
    assert abs(r[0] - np.sqrt(1.25)) < 1e-15
    raw = np.array([[1, 0, 0, 0], [1, 1, 1, 0]], float)[:, :, None]
    assert abs(dg.psrf(raw)[0] - np.sqrt(1.25)) < 1e-15
    rng = np.random.default_rng(2)
    iid = (rng.random((10, 5000, 50)) < 0.3).astype(float)
    r2 = dg.psrf(iid)
    assert (r2 < 1.005).all() and np.allclose(r2, dg.psrf_binary(iid.mean(axis=1), 5000))
    assert dg.psrf_binary(np.array([[0.0], [1.0]]), 10)[0] == np.inf
    assert dg.psrf_binary(np.array([[1.0], [1.0]]), 10)[0] == 1.0


def test_mixing_time_is_first_point_after_which_all_stay_below():
    t = [10, 20, 30, 40, 50]
    assert dg.mixing_time(t, [1.5, 1.0, 1.02, 1.005, 1.001]) == 40
    assert dg.mixing_time(t, [1.0, 1.0, 1.0, 1.0, 1.0]) == 10
    assert dg.mixing_time(t, [1.0, 1.0, 1.0, 1.0, 1.2]) is None
