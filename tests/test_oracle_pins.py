"""Pins of the oracle against things other than itself: the paper's printed
equation, closed forms, invariants, library routines and brute force.

Each test names the mistake in the oracle it is there to catch."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.stats

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- delays

def test_delays_match_paper_eq1_printed_form():
    """Chapter 1, Eq. (1) with its printed constant (ms, GHz) against the
    oracle (s, MHz, 7-digit constant). Catches a wrong unit, a wrong power of
    the frequency or a swapped frequency difference."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "eq1_worked_delays.txt"))
            if l.strip() and not l.startswith("#")]
    for nu1, nu2, dm, dt_ms, ts_ms in rows:
        f = [float(nu2) * 1e3, float(nu1) * 1e3]          # MHz, top first
        d = oracle.delay_table(f, [float(dm)], float(ts_ms) * 1e-3)
        assert d[0, 0] == 0
        exact = float(dt_ms) / float(ts_ms)
        assert abs(d[0, 1] - exact) <= 0.5 + 1e-3, (nu1, nu2, dm, d[0, 1], exact)
        # away from a rounding tie the two constants must agree exactly
        if abs((exact % 1.0) - 0.5) > 0.01:
            assert d[0, 1] == math.floor(exact + 0.5)


def test_delays_match_exact_rational_evaluation():
    """The FP64 delay equals the exactly-rounded rational value of the same law
    except within 1e-9 of a tie. Catches a wrong evaluation order that costs
    more than rounding noise, a wrong constant or a dropped decimation."""
    K = Fraction("4148.808")
    freqs = np.linspace(750.0, 550.0, 257)
    dms = np.linspace(0.0, 1000.0, 37)
    for dec in (1, 4):
        d = oracle.delay_table(freqs, dms, 81.92e-6, dec)
        ft = Fraction(float(freqs.max()))
        for i, dm in enumerate(dms):
            for c in range(0, 257, 16):
                f = Fraction(float(freqs[c]))
                v = K * Fraction(float(dm)) * (1 / (f * f) - 1 / (ft * ft)) / (dec * Fraction(81.92e-6))
                fl = math.floor(v + Fraction(1, 2))
                if abs(v - math.floor(v) - Fraction(1, 2)) > Fraction(1, 10**9):
                    assert d[i, c] == fl, (dec, dm, c)


def test_delay_invariants_tiny_and_full_band():
    """Zero at DM 0 and at the top channel; non-decreasing in DM and as the
    frequency falls; never negative. Catches a wrong reference frequency or
    a sign error (R2)."""
    for f, ts, dms in [(np.linspace(500, 300, 256), 1.31072e-3, np.arange(201.0)),
                       (np.linspace(750, 550, 4096), 81.92e-6, np.linspace(0, 1000, 64))]:
        d = oracle.delay_table(f, dms, ts)
        assert (d[0] == 0).all()
        assert (d[:, 0] == 0).all()
        assert (np.diff(d, axis=0) >= 0).all()
        assert (np.diff(d, axis=1) >= 0).all()
    # unsorted frequencies: reference is the max listed frequency
    f = np.array([400.0, 500.0, 300.0, 450.0])
    d = oracle.delay_table(f, [100.0], 1e-3)
    assert d[0, 1] == 0 and d[0, 2] > d[0, 0] > d[0, 3] > 0


def test_delay_values_tiny():
    """The tiny workload: bottom channel at DM 100 is 2251 samples (Eq. (1)
    with the printed constant gives 2950.26 ms / 1.31072 ms = 2250.8) and the
    maximum delay at DM 200 is 4502."""
    f = np.linspace(500.0, 300.0, 256)
    d = oracle.delay_table(f, np.arange(201.0), 1.31072e-3)
    assert d[100, 255] == 2251
    assert d[100, 1] == 4
    assert d.max() == 4502


def test_delay_rounds_half_up():
    """R3: an exact .5 rounds up (round-half-even would give 2 here)."""
    dm = 4.0 / oracle.K_DM
    for _ in range(64):
        if oracle.K_DM * dm == 4.0:
            break
        dm = float(np.nextafter(dm, 1.0 if oracle.K_DM * dm < 4.0 else 0.0))
    assert oracle.K_DM * dm == 4.0
    # diff = 1/1 - 1/16 = 0.9375; v = 4 * 0.9375 / 1.5 = 2.5 exactly
    d = oracle.delay_table([4.0, 1.0], [dm], 1.5)
    assert d[0, 1] == 3


def test_dm_range_values():
    """R10: count = round((hi-lo)/step), DM_i = lo + i*step (not cumulative)."""
    v = oracle.dm_range_values(0.0, 100.0, 0.1)
    assert len(v) == 1000 and v[0] == 0.0 and v[3] == 3 * 0.1
    counts = [len(oracle.dm_range_values(lo, hi, st)) for lo, hi, st, _ in synth.MULTI_RANGES]
    assert counts == [1000, 1000, 800, 800, 750]


# ---------------------------------------------------------------- dedispersion

def _brute(x, delays, length):
    """Explicit per-sample triple loop in pure Python."""
    ndm, nchan = delays.shape
    out = [[0] * length for _ in range(ndm)]
    xl = x.tolist()
    for i in range(ndm):
        for j in range(length):
            s = 0
            for c in range(nchan):
                s += xl[c][j + int(delays[i][c])]
            out[i][j] = s
    return np.array(out, dtype=np.int64)


def test_dedisperse_equals_explicit_triple_loop():
    """P3: catches a transposed delay table, a reversed shift or a dropped
    channel."""
    rng = _rng(5)
    for nchan, T, ndm in [(1, 40, 1), (7, 120, 5), (16, 256, 8)]:
        f = np.sort(rng.uniform(300, 500, nchan))[::-1]
        dms = np.sort(rng.uniform(0, 10, ndm))
        d = oracle.delay_table(f, dms, 5e-3)
        L = T - int(d.max())
        assert L > 0
        x = rng.integers(0, 256, (nchan, T), dtype=np.uint8)
        np.testing.assert_array_equal(oracle.dedisperse(x, d, L), _brute(x, d, L))


def test_dm0_is_column_sum():
    """P1: at DM 0 the plane row is the plain channel sum."""
    rng = _rng(6)
    x = rng.integers(0, 256, (64, 500), dtype=np.uint8)
    f = np.linspace(500, 300, 64)
    d = oracle.delay_table(f, [0.0, 10.0], 1e-3)
    y = oracle.dedisperse(x, d, 500 - int(d.max()))
    np.testing.assert_array_equal(y[0], x.astype(np.int64).sum(axis=0)[: y.shape[1]])


def test_impulse_bow_tie():
    """P4: a single non-zero sample v at (c0, u) lands at j = u - delay(c0, i)
    in every DM row and nowhere else. Catches j - delay vs j + delay."""
    f = np.linspace(500, 300, 32)
    dms = np.arange(0.0, 50.0, 2.0)
    d = oracle.delay_table(f, dms, 1e-3)
    T = 2000
    L = T - int(d.max())
    x = np.zeros((32, T), dtype=np.uint8)
    c0, u = 29, 1500
    x[c0, u] = 77
    y = oracle.dedisperse(x, d, L)
    for i in range(len(dms)):
        j = u - d[i, c0]
        expect = np.zeros(L, dtype=np.int64)
        if 0 <= j < L:
            expect[j] = 77
        np.testing.assert_array_equal(y[i], expect)


def test_linearity_and_shift_equivariance():
    """P5: y(a + b) = y(a) + y(b); shifting the input by s shifts the plane."""
    rng = _rng(7)
    f = np.linspace(500, 300, 24)
    d = oracle.delay_table(f, np.arange(0.0, 40.0, 4.0), 5e-3)
    T = 900
    L = T - int(d.max()) - 10
    a = rng.integers(0, 120, (24, T), dtype=np.uint8)
    b = rng.integers(0, 120, (24, T), dtype=np.uint8)
    np.testing.assert_array_equal(oracle.dedisperse(a + b, d, L),
                                  oracle.dedisperse(a, d, L) + oracle.dedisperse(b, d, L))
    s = 10
    ys = oracle.dedisperse(a[:, s:], d, L)
    np.testing.assert_array_equal(ys, oracle.dedisperse(a, d, L + s)[:, s:])


def test_pulse_only_plane_tiny():
    """P6: the tiny workload's pulse alone gives exactly 40*256 = 10240 on
    [3000, 3004) at DM 100 and less everywhere at other DM trials."""
    w = synth.tiny(oracle.delay_table, with_data=False)
    d = oracle.delay_table(w.freqs_mhz, w.dm_list, w.t_samp)
    x = np.zeros((256, w.nsamp), dtype=np.uint8)
    p = w.pulses[0]
    synth.inject_pulse(x, oracle.delay_table(w.freqs_mhz, [p.dm], w.t_samp)[0],
                       p.t0, p.width, p.amp)
    L = w.nsamp - int(d.max())
    rows = [98, 99, 100, 101, 102]
    y = oracle.dedisperse_rows(x, d, rows, L)
    np.testing.assert_array_equal(y[2, 3000:3004], [10240] * 4)
    assert y[2].max() == 10240 and np.count_nonzero(y[2] == 10240) == 4
    for k in (0, 1, 3, 4):
        assert y[k].max() < 10240


def test_constant_input_has_no_candidates():
    """P7: constant input gives y = C*v*dec, sigma 0, all S/N 0, no candidate."""
    plan = oracle.make_plan(np.linspace(500, 300, 16), 1e-3,
                            ranges=[(0.0, 20.0, 5.0, 1), (20.0, 40.0, 5.0, 2)],
                            widths=[1, 2, 4], cand_block=64, threshold=-1.0)
    T = plan.overlap + 300
    x = np.full((16, T), 9, dtype=np.uint8)
    for r, (rows, y, res) in enumerate(oracle.run(plan, x)):
        dec = plan.ranges[r].dec
        assert (y == 16 * 9 * dec).all()
        for rr in res:
            assert rr.std == 0.0 and rr.cands == [] and rr.best[0] == 0.0


def test_decimation_consistency_dm0():
    """P9: at DM 0, the decimated plane equals the full-rate plane summed in
    groups of dec aligned to sample 0."""
    rng = _rng(8)
    x = rng.integers(0, 256, (8, 1003), dtype=np.uint8)
    f = np.linspace(500, 300, 8)
    y1 = oracle.dedisperse(x, oracle.delay_table(f, [0.0], 1e-3), 1000)[0]
    for dec in (2, 4, 8):
        yd = oracle.dedisperse(oracle.decimate(x, dec),
                               oracle.delay_table(f, [0.0], 1e-3, dec), 1000 // dec)[0]
        np.testing.assert_array_equal(yd, y1[: (1000 // dec) * dec].reshape(-1, dec).sum(1))
    # a hand example of the grouping itself
    np.testing.assert_array_equal(oracle.decimate(np.array([[1, 2, 3, 4, 5]]), 2), [[3, 7]])


# ---------------------------------------------------------------- search

def test_boxcar_matches_convolution_and_prefix_identity():
    """P8: B_w equals numpy's 'valid' convolution with a ones kernel and
    P[j+w] - P[j] of the prefix sum. Catches an off-by-one window."""
    rng = _rng(9)
    y = rng.integers(0, 10**6, 700).astype(np.int64)
    n = 600
    P = np.concatenate([[0], np.cumsum(y)])
    for w in (1, 2, 3, 16, 64, 101):
        b = oracle.boxcar_sums(y, w, n)
        np.testing.assert_array_equal(b, np.convolve(y, np.ones(w, dtype=np.int64), "valid")[:n])
        np.testing.assert_array_equal(b, P[w:w + n] - P[:n])


def test_moments_match_numpy_population_stats():
    """R7: mean / population std against numpy (ddof=0). Catches ddof=1 or a
    missing square root."""
    rng = _rng(10)
    for n in (2, 37, 5000):
        y = rng.integers(0, 2 * 10**6, n + 5).astype(np.int64)
        s1, s2 = oracle.row_moments(y, n)
        assert s1 == int(y[:n].sum()) and s2 == sum(int(v) ** 2 for v in y[:n])
        mu, sg = oracle.mean_sigma(s1, s2, n)
        assert mu == pytest.approx(np.mean(y[:n]), rel=1e-15)
        assert sg == pytest.approx(np.std(y[:n].astype(np.float64)), rel=1e-9)


def test_width1_snr_is_zscore():
    """P8 second half: at width 1 the S/N is scipy's z-score (ddof=0)."""
    rng = _rng(11)
    y = rng.integers(1000, 5000, 4000).astype(np.int64)
    n = 4000
    mu, sg = oracle.mean_sigma(*oracle.row_moments(y, n), n)
    s = oracle.snr_matrix(y, [1], n, mu, sg)[:, 0]
    np.testing.assert_allclose(s, scipy.stats.zscore(y.astype(np.float64)), rtol=1e-9, atol=1e-12)


def test_noise_snr_is_unit_normal_per_width():
    """P11 (statistical sanity): on white Gaussian noise every width gives
    S/N with mean ~0 and std ~1. Catches a missing or wrong sqrt(w)."""
    rng = _rng(12)
    n = 200000
    y = np.rint(rng.normal(50000.0, 300.0, n + 63)).astype(np.int64)
    mu, sg = oracle.mean_sigma(*oracle.row_moments(y, n), n)
    s = oracle.snr_matrix(y, [1, 4, 16, 64], n, mu, sg)
    assert np.all(np.abs(s.mean(axis=0)) < 0.05)
    assert np.all(np.abs(s.std(axis=0) - 1.0) < 0.05)


def _brute_search(y, widths, n, cb, thr):
    ys = [int(v) for v in y]
    s1 = sum(ys[:n]); s2 = sum(v * v for v in ys[:n])
    mu = s1 / n
    var = Fraction(n * s2 - s1 * s1, n * n)
    sg = math.sqrt(var)
    best = None
    cells = []
    for j0 in range(0, n, cb):
        cb_best = None
        for j in range(j0, min(j0 + cb, n)):
            for w in widths:
                b = sum(ys[j:j + w])
                s = (b - w * mu) / (sg * math.sqrt(w))
                if cb_best is None or s > cb_best[0]:
                    cb_best = (s, j, w)
        cells.append(cb_best)
        if best is None or cb_best[0] > best[0]:
            best = cb_best
    return best, [c for c in cells if c[0] > thr]


def test_search_row_equals_brute_force():
    """R6-R9 against loops written out per window: per-DM best, cell
    candidates, first-maximum tie order and the strict threshold."""
    rng = _rng(13)
    for n, cb in [(50, 16), (300, 64), (257, 256)]:
        y = rng.integers(0, 50, n + 15).astype(np.int64)
        y[n // 3: n // 3 + 4] += 60
        widths = [1, 2, 4, 8, 16]
        rr = oracle.search_row(y, widths, n, cb, 2.5)
        best, cands = _brute_search(y, widths, n, cb, 2.5)
        assert rr.best[1:] == best[1:] and rr.best[0] == pytest.approx(best[0], rel=1e-12)
        assert [c[1:] for c in rr.cands] == [c[1:] for c in cands]
        for a, b in zip(rr.cands, cands):
            assert a[0] == pytest.approx(b[0], rel=1e-12)
    # tie order: two identical pulses -> the earlier one wins; equal S/N
    # across widths cannot arise from distinct sums so only j order matters
    y = np.zeros(120, dtype=np.int64)
    y[10] = y[70] = 100
    y[40] = 1
    rr = oracle.search_row(y, [1, 2], 100, 100, 0.0)
    # width 1 at j=10 and j=70 tie exactly (width 2 scores lower): first wins
    assert rr.best[1:] == (10, 1)
    # strict threshold: a threshold equal to the best S/N drops that cell
    rr2 = oracle.search_row(y, [1, 2], 100, 100, rr.best[0])
    assert rr2.cands == []


def test_tiny_workload_recovers_injected_pulse():
    """Injection recovery (Section 2.4 method): the best candidate over all
    DM trials of the tiny workload is DM 100, sample 3000, width 4."""
    w = synth.tiny(oracle.delay_table)
    plan = oracle.make_plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths,
                            cand_block=w.cand_block, threshold=w.threshold)
    assert plan.overlap == 4502 + 15
    assert plan.owned(w.nsamp) == [8192 - 4517]
    rows = list(range(90, 111))
    (rr, y, res), = oracle.run(plan, w.x, rows=[rows])
    assert y.shape == (21, 3690)
    k = int(np.argmax([r.best[0] for r in res]))
    assert rows[k] == 100
    assert res[k].best[1:] == (3000, 4)
    assert res[k].best[0] > 20.0


def test_plane_checksums_equal_brute_force_sums():
    """The prefix-sum checksums of every plane row equal the row sum and the
    index-weighted row sum of the explicit per-sample triple loop (catches an
    off-by-one in the prefix bounds, a missing delay term in the weighted sum
    or a transposed delay table); uint16 rows of a decimated range too."""
    rng = _rng(17)
    for nchan, T, ndm, hi in [(1, 30, 1, 255), (7, 150, 6, 255), (16, 300, 9, 4080)]:
        f = np.sort(rng.uniform(300, 500, nchan))[::-1]
        dms = np.sort(rng.uniform(0, 12, ndm))
        d = oracle.delay_table(f, dms, 5e-3)
        L = T - int(d.max())
        x = rng.integers(0, hi + 1, (nchan, T)).astype(np.uint8 if hi == 255 else np.uint16)
        y = _brute(x, d, L)
        a, b = oracle.plane_checksums(x, d, L)
        j = np.arange(L)
        assert a.tolist() == [int(sum(int(v) for v in row)) for row in y]
        assert b.tolist() == [int(sum(int(k) * int(v) for k, v in zip(j, row))) for row in y]


def test_plane_checksums_closed_form_constant_input():
    """Constant input v: every row is nchan*v over `length` samples, so the
    checksums are nchan*v*L and nchan*v*L*(L-1)/2 at every trial."""
    f = np.linspace(750, 550, 33)
    d = oracle.delay_table(f, np.linspace(0, 40, 11), 81.92e-6)
    L = 5000
    x = np.full((33, L + int(d.max())), 201, dtype=np.uint8)
    a, b = oracle.plane_checksums(x, d, L)
    assert (a == 33 * 201 * L).all() and (b == 33 * 201 * L * (L - 1) // 2).all()
