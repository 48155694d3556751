"""RFI pre-conditioning of one chunk before dedispersion, as the paper's RFI
tool is described (Section 2.1 and its figure of the tool's steps): the
average spectrum (mean intensity of each channel), its moving median over 21
channels as the bandpass, channels that are > 4 sigma outliers of the
bandpass-corrected spectrum flagged, the frequency-averaged time series over
the unflagged channels, time samples that are > 3 sigma outliers of it
flagged, the time- and frequency-domain flagging done twice.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the description gives no estimator or data format details):
  P1  Channel mean m_c = (sum over unflagged samples of x[c][t]) / (their
      count), FP64 of the exact integer sum (all samples in the first round
      or when every sample is flagged).
  P2  Bandpass b_c = median of m over channels [c - h, c + h] clipped to the
      band, window 2h + 1 (21); medians are lower medians (element
      (n - 1) // 2 of the sorted values) throughout.
  P3  Residual spectrum r = m - b (FP64). sigma = 1.4826 * MAD, MAD the lower
      median of |v - median(v)|. Channel c is flagged when
      |r_c - median(r)| > k_chan * sigma_r (k_chan = 4.0); sigma 0 flags none.
  P4  Zero-DM series z_t = sum of x[c][t] over unflagged channels (exact
      integer); sample t is flagged when |z_t - median(z)| > k_time * sigma_z
      (k_time = 3.0; medians over all samples); sigma 0 flags none.
  P5  Rounds: P1-P4 twice; each round recomputes the channel flags from the
      spectrum of the samples unflagged by the previous round, then the time
      flags from the channels it flags. The last round's flags are the result.
  P6  Output as exact integer maps: a per-channel table lut[c][v] =
      0 for a flagged channel, else clip(v - B_c + L, 0, 255) with
      B_c = floor(b_c + 0.5) and L = floor(median(b) + 0.5) (bandpass
      subtracted, every channel re-centred on the median level); and a time
      mask (1 = keep). The pre-conditioned chunk is
      x'[c][t] = mask[t] ? lut[c][x[c][t]] : 0.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

__all__ = ["lower_median", "robust_sigma", "running_median", "rfi_estimate", "precondition"]

MAD_SCALE = 1.4826


def lower_median(v) -> float:
    """Element (n - 1) // 2 of the sorted values (P2)."""
    s = np.sort(np.asarray(v), kind="stable")
    return s[(len(s) - 1) // 2]


def robust_sigma(v) -> Tuple[float, float]:
    """(median, 1.4826 * MAD) with lower medians (P3)."""
    v = np.asarray(v)
    med = lower_median(v)
    mad = lower_median(np.abs(v - med))
    return med, MAD_SCALE * float(mad)


def running_median(m: np.ndarray, window: int) -> np.ndarray:
    """Moving lower median over [c - h, c + h] clipped to the band (P2)."""
    h = window // 2
    n = len(m)
    return np.array([lower_median(m[max(0, c - h):min(n, c + h + 1)]) for c in range(n)],
                    dtype=np.float64)


def rfi_estimate(x: np.ndarray, window: int = 21, rounds: int = 2, k_chan: float = 4.0,
                 k_time: float = 3.0):
    """Channel flags, time flags, bandpass, lut [C][256] uint8 and time mask
    [T] uint8 of a channel-major uint8 chunk x[c][t] (P1-P6)."""
    C, T = x.shape
    xi = x.astype(np.int64)
    tflag = np.zeros(T, dtype=bool)
    cflag = np.zeros(C, dtype=bool)
    b = np.zeros(C)
    for _ in range(rounds):
        keep_t = ~tflag
        if keep_t.sum() == 0:
            keep_t = np.ones(T, dtype=bool)
        nt = int(keep_t.sum())
        m = np.array([float(int(xi[c, keep_t].sum())) / float(nt) for c in range(C)])
        b = running_median(m, window)
        r = m - b
        mr, sr = robust_sigma(r)
        cflag = (np.abs(r - mr) > k_chan * sr) if sr > 0.0 else np.zeros(C, dtype=bool)
        z = xi[~cflag].sum(axis=0)
        mz, sz = robust_sigma(z)
        tflag = (np.abs(z - mz).astype(np.float64) > k_time * sz) if sz > 0.0 \
            else np.zeros(T, dtype=bool)
    B = np.floor(b + 0.5).astype(np.int64)
    L = int(math.floor(float(lower_median(b)) + 0.5))
    v = np.arange(256, dtype=np.int64)
    lut = np.clip(v[None, :] - B[:, None] + L, 0, 255).astype(np.uint8)
    lut[cflag] = 0
    mask = (~tflag).astype(np.uint8)
    return cflag, tflag, b, lut, mask


def precondition(x: np.ndarray, lut: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """x'[c][t] = mask[t] ? lut[c][x[c][t]] : 0 (P6)."""
    out = np.take_along_axis(lut, x.astype(np.int64), axis=1)
    out[:, mask == 0] = 0
    return out.astype(np.uint8)
