"""Pins of the FFA oracle (folding transform, trial periods and the boxcar
search of folded profiles) against closed forms, invariants and brute force."""
import math

import numpy as np
import pytest

import oracle


def _shifts(m: int, p: int) -> np.ndarray:
    """delta[i][s]: the circular shift that profile s applies to row i, read
    from the transform of one-hot stacks (each must give a single 1)."""
    d = np.zeros((m, m), dtype=np.int64)
    for i in range(m):
        rows = np.zeros((m, p), dtype=np.int64)
        rows[i, 0] = 1
        T = oracle.ffa_transform(rows)
        for s in range(m):
            nz = np.nonzero(T[s])[0]
            assert len(nz) == 1 and T[s, nz[0]] == 1, (m, i, s)
            d[i, s] = (-nz[0]) % p
    return d


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 13, 64])
def test_zero_trial_is_the_plain_fold_and_totals_are_kept(m):
    g = np.random.Generator(np.random.PCG64(m))
    rows = g.integers(0, 1000, (m, 37))
    T = oracle.ffa_transform(rows)
    assert np.array_equal(T[0], rows.sum(axis=0))
    assert np.all(T.sum(axis=1) == rows.sum())


@pytest.mark.parametrize("m", [2, 3, 5, 7, 8, 16, 33])
def test_last_trial_drifts_one_bin_per_row(m):
    g = np.random.Generator(np.random.PCG64(100 + m))
    p = 29
    rows = g.integers(0, 1000, (m, p))
    want = np.zeros(p, dtype=np.int64)
    for i in range(m):
        for j in range(p):
            want[j] += rows[i][(j + i) % p]
    assert np.array_equal(oracle.ffa_transform(rows)[m - 1], want)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_power_of_two_stack_is_the_classic_ffa(k):
    """For m = 2^k each level of the classic FFA adds the shift
    ceil(floor(s / 2^r) / 2) to the rows whose bit k-1-r is set, so row i of
    profile s is shifted by the sum of those terms."""
    m = 1 << k
    d = _shifts(m, 2 * m + 1)
    for i in range(m):
        for s in range(m):
            want = sum(((s >> r) + 1) // 2 for r in range(k) if (i >> (k - 1 - r)) & 1)
            assert d[i, s] == want, (m, i, s)


@pytest.mark.parametrize("m", [3, 5, 6, 9, 12, 17, 31, 33, 100])
def test_any_height_is_a_sum_of_shifted_rows_near_the_linear_drift(m):
    """Every profile takes each row exactly once; the first row is never
    shifted, the last by exactly s; shifts grow with the row and the trial
    and stay within half a bin per recursion level of i s / (m - 1)."""
    d = _shifts(m, 2 * m + 3)
    ideal = np.arange(m)[:, None] * np.arange(m)[None, :] / (m - 1)
    assert np.all(d[0] == 0) and np.array_equal(d[-1], np.arange(m))
    assert np.all(np.diff(d, axis=0) >= 0) and np.all(np.diff(d, axis=1) >= 0)
    assert np.abs(d - ideal).max() <= math.ceil(math.log2(m)) / 2


def test_linear_in_the_input():
    g = np.random.Generator(np.random.PCG64(7))
    a = g.integers(0, 500, (11, 23))
    b = g.integers(0, 500, (11, 23))
    assert np.array_equal(oracle.ffa_transform(a + 3 * b),
                          oracle.ffa_transform(a) + 3 * oracle.ffa_transform(b))


def test_trial_periods_span_p_to_p2_over_p_minus_1():
    p, m, tau = 250, 64, 1e-3
    per = oracle.trial_periods(p, m, tau)
    f = oracle.trial_frequencies(p, m, tau)
    assert per[0] == pytest.approx(p * tau) and per[-1] == pytest.approx(p * p / (p - 1) * tau)
    assert np.allclose(f * per, 1.0)
    assert np.allclose(np.diff(f), -1.0 / ((m - 1) * p * p * tau))
    assert oracle.trial_periods(p, 1, tau)[0] == p * tau


def test_boxcar_sums_brute_force():
    prof = np.array([5, 1, 4, 1, 5, 9, 2, 6], dtype=np.int64)
    for w in range(1, 8):
        got = oracle.circular_boxcar_sums(prof, w)
        want = [sum(prof[(j + k) % 8] for k in range(w)) for j in range(8)]
        assert list(got) == want


def test_noise_profiles_have_unit_snr_spread():
    """White noise: every folded bin sums m independent samples, so the S/N
    of w adjacent bins has mean 0 and, as the bins sum to the fixed total,
    deviation sqrt(1 - w/p). Disjoint windows of independent series."""
    g = np.random.Generator(np.random.PCG64(21))
    p = 128
    vals = {1: [], 8: []}
    for _ in range(128):
        y = np.round(g.normal(1000.0, 30.0, 1 << 14)).astype(np.int64)
        T = oracle.ffa_transform(oracle.stack_rows(y, p))
        n, s1, s2, mu, sigma = oracle.fold_moments(y, p)
        assert n == 1 << 14 and s1 == int(y.sum()) and s2 == int((y * y).sum())
        for w in vals:
            vals[w].append(oracle.profile_snr(T[37], [w], T.shape[0], mu, sigma)[0][::w])
    for w, v in vals.items():
        v = np.concatenate(v)
        assert abs(v.mean()) < 0.06 and abs(v.std() / math.sqrt(1 - w / p) - 1.0) < 0.06, \
            (w, v.mean(), v.std())


@pytest.mark.parametrize("s0", [0, 17, 40, 63])
def test_pulse_train_peaks_at_its_trial(s0):
    """A pulse train whose period drifts s0 bins over the stack is found in
    profile s0 (or a neighbour), far above the other trials."""
    g = np.random.Generator(np.random.PCG64(s0))
    p, m = 200, 64
    y = np.round(g.normal(100.0, 10.0, m * p + 50)).astype(np.int64)
    P = p + s0 / (m - 1)
    for i in range(m):
        t = int(round(30 + i * P))
        y[t:t + 4] += 12
    T, mom, best = oracle.ffa_search(y, p, [1, 2, 4, 8])
    snr = np.array([b[0] for b in best])
    k = int(np.argmax(snr))
    assert abs(k - s0) <= 1, (k, s0)
    assert snr[k] > 15.0 and snr[k] > 2.0 * np.median(snr)
    assert abs(best[k][1] - 30) <= 3


def test_degenerate_constant_series_and_single_row():
    T, mom, best = oracle.ffa_search(np.full(1000, 7), 100, [1, 3])
    assert mom[4] == 0.0 and all(b == (0.0, 0, 1) for b in best)
    y = np.arange(50)
    T, mom, best = oracle.ffa_search(y, 40, [1, 2])
    assert T.shape == (1, 40) and np.array_equal(T[0], np.arange(40))
    assert best[0][1:] == (38, 2)
    with pytest.raises(ValueError):
        oracle.ffa_search(y, 40, [40])
