"""Pins of the RFI pre-conditioning oracle: its medians against scipy, and
its flags and bandpass correction on filterbanks with planted RFI."""
import numpy as np

import oracle
import synth
from oracle.rfi import MAD_SCALE, lower_median, precondition, rfi_estimate, robust_sigma, \
    running_median


def test_running_median_interior_equals_scipy_median_filter():
    from scipy.ndimage import median_filter
    g = np.random.Generator(np.random.PCG64(1))
    m = g.normal(100.0, 5.0, 500)
    ours = running_median(m, 21)
    ref = median_filter(m, size=21)
    assert np.array_equal(ours[10:-10], ref[10:-10])
    # clipped edge windows: c = 0 uses m[0:11]
    assert ours[0] == np.sort(m[:11])[5]


def test_robust_sigma_equals_numpy_and_scipy_for_odd_counts():
    from scipy.stats import median_abs_deviation
    g = np.random.Generator(np.random.PCG64(2))
    v = g.normal(0.0, 3.0, 1001)
    med, sig = robust_sigma(v)
    assert med == np.median(v)
    assert sig == MAD_SCALE * median_abs_deviation(v, scale=1.0)
    # lower median for an even count
    assert lower_median([4, 1, 3, 2]) == 2


def _rfi_chunk(seed=5, C=256, T=4096):
    x = synth.filterbank(seed, C, T, 100.0, 10.0).astype(np.int64)
    shape = (20.0 * np.sin(np.linspace(0, 3, C))).round().astype(np.int64)  # bandpass
    x += shape[:, None]
    bad_ch = [17, 90, 91, 200]
    x[bad_ch] += 60                     # narrowband RFI
    bad_t = [100, 101, 2500, 3900]
    x[:, bad_t] += 40                   # broadband bursts
    return np.clip(x, 0, 255).astype(np.uint8), shape, bad_ch, bad_t


def test_flags_find_planted_rfi_and_little_else():
    x, shape, bad_ch, bad_t = _rfi_chunk()
    cflag, tflag, b, lut, mask = rfi_estimate(x)
    assert set(bad_ch) <= set(np.nonzero(cflag)[0].tolist())
    assert set(bad_t) <= set(np.nonzero(tflag)[0].tolist())
    # a few band-edge channels, where the clipped median window lags the
    # bandpass slope, may be flagged too
    assert cflag.sum() <= len(bad_ch) + x.shape[0] // 16
    assert tflag.sum() <= len(bad_t) + 0.01 * x.shape[1]   # ~0.3% of Gaussian noise is > 3 sigma
    assert (lut[cflag] == 0).all() and (mask == (~tflag).astype(np.uint8)).all()


def test_bandpass_correction_recentres_channels():
    x, shape, bad_ch, _ = _rfi_chunk()
    cflag, tflag, b, lut, mask = rfi_estimate(x)
    y = precondition(x, lut, mask)
    L = int(np.floor(lower_median(b) + 0.5))
    good = ~cflag
    means = y[good][:, mask == 1].mean(axis=1)
    # each kept channel's mean sits within a fraction of a count of L, up to the
    # residual of the 21-channel median bandpass itself
    assert np.abs(means - L).max() < 2.0
    assert (y[cflag] == 0).all() and (y[:, mask == 0] == 0).all()


def test_identity_maps_and_zero_dm_row():
    x = synth.filterbank(8, 64, 1000, 120.0, 20.0)
    ident = np.tile(np.arange(256, dtype=np.uint8), (64, 1))
    assert np.array_equal(precondition(x, ident, np.ones(1000, np.uint8)), x)
    _, _, _, lut, mask = rfi_estimate(x)
    y = precondition(x, lut, mask)
    # DM 0 of the pre-conditioned chunk is its column sum
    d = oracle.delay_table(np.linspace(500, 300, 64), [0.0], 1e-3)
    row = oracle.dedisperse(y, d, 1000)[0]
    assert np.array_equal(row, y.astype(np.int64).sum(axis=0))


def test_constant_data_flags_nothing():
    x = np.full((32, 500), 77, dtype=np.uint8)
    cflag, tflag, b, lut, mask = rfi_estimate(x)
    assert not cflag.any() and not tflag.any()
    assert np.array_equal(precondition(x, lut, mask), x)


def hand_case():
    """7 channels x 10 samples, worked by hand in
    test_two_rounds_hand_worked_case: channel baselines
    101, 100, 100, 101, 100, 100, 100; channel 0 adds t mod 2 and channel 1
    adds t mod 3 (so the noise estimates are not zero); channel 5 is hot (+30,
    and +40 more at t = 7); channel 2 has a +100 spike at t = 4; every channel
    gets +10 at t = 4 (a broadband burst)."""
    x = np.array([101, 100, 100, 101, 100, 100, 100], dtype=np.int64)[:, None] + \
        np.zeros((1, 10), dtype=np.int64)
    t = np.arange(10)
    x[0] += t % 2
    x[1] += t % 3
    x[5] += 30
    x[5, 7] += 40
    x[2, 4] += 100
    x[:, 4] += 10
    return x.astype(np.uint8)


def test_two_rounds_hand_worked_case():
    """P1, P4, P5 on a case small enough to work by hand (window 3). Round 2
    must take its channel means over the samples round 1 kept, and the
    zero-DM series over the channels of its own round only:

    Round 1 (all 10 samples). Channel sums 1025, 1019, 1110, 1020, 1010,
    1350, 1010, so m = 102.5, 101.9, 111, 102, 101, 135, 101. Lower medians of
    3-channel windows (2 at the edges): b = 101.9, 102.5, 102, 102, 102, 101,
    101; r = m - b = 0.6, -0.6, 9, 0, -1, 34, 0; median(r) = 0, MAD = 0.6,
    4 sigma = 4 * 1.4826 * 0.6 = 3.558: channels 2 and 5 flagged. Zero-DM
    series over channels 0, 1, 3, 4, 6: 502, 504, 504, 503, 553, 505, 502, 504,
    504, 503; median 504, MAD 1, 3 sigma = 4.448: sample 4 flagged.

    Round 2 (the 9 samples other than t = 4). Sums 914, 908, 900, 909, 900,
    1210, 900, so m = 101.556, 100.889, 100, 101, 100, 134.444, 100;
    b = 100.889, 100.889, 100.889, 100, 101, 100, 100; r = 0.667, 0, -0.889,
    1, -1, 34.444, 0; median 0, MAD 0.889, 4 sigma = 5.272: only channel 5
    (the spike of channel 2 no longer counts). Zero-DM series over every
    channel but 5: 602, 604, 604, 603, 763, 605, 602, 604, 604, 603; median
    604, MAD 1: sample 4 flagged, sample 7 (channel 5's spike) not.

    Result: channels {5}, samples {4}; bandpass B = floor(b + 0.5) = 101,
    101, 101, 100, 101, 100, 100 and level L = floor(100.889 + 0.5) = 101.
    Round-2 means over all samples would flag channel 2 again; a zero-DM
    series over all channels would flag sample 7 in both rounds."""
    x = hand_case()
    c1, t1, _, _, _ = rfi_estimate(x, window=3, rounds=1)
    assert np.nonzero(c1)[0].tolist() == [2, 5] and np.nonzero(t1)[0].tolist() == [4]
    cflag, tflag, b, lut, mask = rfi_estimate(x, window=3, rounds=2)
    assert np.nonzero(cflag)[0].tolist() == [5]
    assert np.nonzero(tflag)[0].tolist() == [4]
    assert mask.tolist() == [1, 1, 1, 1, 0, 1, 1, 1, 1, 1]
    assert np.floor(b + 0.5).astype(int).tolist() == [101, 101, 101, 100, 101, 100, 100]
    v = np.arange(256)
    assert (lut[5] == 0).all()
    assert lut[3].tolist() == np.clip(v + 1, 0, 255).tolist()       # B = 100, L = 101
    assert lut[0].tolist() == v.tolist()                             # B = 101
    assert abs(b[0] - 908 / 9) < 1e-12 and b[3] == 100.0 and b[4] == 101.0
