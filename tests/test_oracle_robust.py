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


def test_block_baseline_with_unit_blocks_is_the_running_median():
    """D = 1: the baseline is the per-sample running median (window 2h+1,
    clipped at the ends), i.e. scipy's median filter in the interior."""
    from scipy.ndimage import median_filter
    g = np.random.Generator(np.random.PCG64(9))
    y = g.integers(0, 1000, 3000)
    base = oracle.block_baseline(y, 3000, 1, 10)
    ref = median_filter(y, size=21)
    assert np.array_equal(base[10:-10], ref[10:-10])


def test_dereddening_removes_a_slow_baseline_and_keeps_the_pulse():
    g = np.random.Generator(np.random.PCG64(10))
    L = 1 << 14
    t = np.arange(L)
    y = np.round(g.normal(1000.0, 10.0, L) + 200.0 * np.sin(2 * np.pi * t / 6000.0))
    y = y.astype(np.int64)
    y[9000:9008] += 150
    M = 4096 * 255
    d = oracle.dereddened(y, L, 64, 2, M) - M // 2
    # the slow wave is gone (its 200-count swing left within a few counts)
    assert np.abs(np.convolve(d, np.ones(512) / 512, "valid")).max() < 20.0
    plain = oracle.search_row(y, [1, 8], L - 7, 1024, 6.0)
    red = oracle.search_row(y, [1, 8], L - 7, 1024, 6.0, dered=(64, 2, M))
    assert red.best[1:] == (9000, 8)
    assert red.best[0] > 5.0 * plain.best[0] or plain.best[1] != 9000


def test_offset_leaves_every_snr_unchanged():
    """The half-scale offset only moves mu: two full scales large enough that
    the clip never acts give the same S/N, cells and candidates."""
    g = np.random.Generator(np.random.PCG64(11))
    y = g.integers(100, 900, 5000)
    a = oracle.search_row(y, [1, 2, 4], 4997, 512, 3.0, dered=(16, 1, 2000))
    b = oracle.search_row(y, [1, 2, 4], 4997, 512, 3.0, dered=(16, 1, 777777))
    assert a.best[1:] == b.best[1:] and abs(a.best[0] - b.best[0]) < 1e-9
    assert [c[1:] for c in a.cands] == [c[1:] for c in b.cands]


def test_dereddened_clip_bounds():
    """Samples more than M/2 below / above their baseline clip to 0 / M."""
    y = np.full(256, 500, dtype=np.int64)
    y[100] = 0
    y[200] = 1000
    d = oracle.dereddened(y, 256, 64, 1, 600)
    assert d[100] == 0 and d[200] == 600 and d[0] == 300
    assert np.all((d >= 0) & (d <= 600))
