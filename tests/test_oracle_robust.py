"""Pins of the robust noise statistics: sigma clipping against scipy's
sigmaclip, median/MAD against numpy/scipy, and their effect on a bright
pulse."""
import numpy as np

import oracle
from oracle.robust import clipped_moments, median_mad, robust_mean_sigma


def test_clipping_to_convergence_equals_scipy_sigmaclip():
    from scipy.stats import sigmaclip
    g = np.random.Generator(np.random.PCG64(1))
    y = np.round(g.normal(1000.0, 30.0, 20001)).astype(np.int64)
    y[::997] += 600                      # outliers
    cnt, s1, s2, mu, sigma = clipped_moments(y, len(y), 3.0, 60)
    kept, lo, hi = sigmaclip(y.astype(np.float64), 3.0, 3.0)
    assert cnt == len(kept) and s1 == int(kept.sum())
    assert abs(mu - kept.mean()) < 1e-9 and abs(sigma - kept.std()) < 1e-9


def test_clipping_with_a_huge_k_is_the_plain_statistics():
    g = np.random.Generator(np.random.PCG64(2))
    y = g.integers(0, 5000, 3001)
    mu0, s0 = oracle.mean_sigma(*oracle.row_moments(y, 3001), 3001)
    cnt, s1, s2, mu, sigma = clipped_moments(y, 3001, 1e9, 5)
    assert cnt == 3001 and mu == mu0 and sigma == s0
    assert robust_mean_sigma(y, 3001, None) == (mu0, s0)


def test_median_mad_equals_numpy_and_scipy():
    from scipy.stats import median_abs_deviation
    g = np.random.Generator(np.random.PCG64(3))
    y = g.integers(0, 100000, 10001)
    med, sig = median_mad(y, len(y))
    assert med == np.median(y)
    assert sig == 1.4826 * median_abs_deviation(y, scale=1.0)
    # lower medians for an even count
    assert median_mad(np.array([1, 2, 3, 10]), 4) == (2.0, 1.4826 * 1.0)


def test_robust_sigma_ignores_a_bright_pulse():
    g = np.random.Generator(np.random.PCG64(4))
    y = np.round(g.normal(500.0, 10.0, 50000)).astype(np.int64)
    y[20000:20050] += 400                 # bright 50-sample pulse
    _, plain = oracle.mean_sigma(*oracle.row_moments(y, len(y)), len(y))
    _, clip = robust_mean_sigma(y, len(y), ("clip", 3.0, 3))
    _, mad = robust_mean_sigma(y, len(y), ("mad",))
    assert plain > 12.0                   # inflated by the pulse
    assert abs(clip - 10.0) < 0.5 and abs(mad - 10.0) < 0.5


def test_search_row_uses_the_chosen_statistics():
    g = np.random.Generator(np.random.PCG64(5))
    y = np.round(g.normal(200.0, 5.0, 4100)).astype(np.int64)
    y[1000:1004] += 60
    base = oracle.search_row(y, [1, 2, 4], 4097, 1024, 6.0)
    rob = oracle.search_row(y, [1, 2, 4], 4097, 1024, 6.0, stats=("mad",))
    assert (base.s1, base.s2) == (rob.s1, rob.s2)
    assert rob.best[1:] == base.best[1:] == (1000, 4)
    med, sig = median_mad(y, 4097)
    assert rob.mean == med and rob.std == sig
