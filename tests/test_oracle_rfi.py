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
