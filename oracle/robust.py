"""Robust noise statistics of a dedispersed series for the S/N of the
single-pulse search: a bright pulse inflates the plain standard deviation, so
the mean and width of the noise can instead come from sigma-clipped moments
or from the median and the median absolute deviation (the paper prefers the
median as the less outlier-sensitive noise estimate, Section 3.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings:
  Q1  Clipped moments: start from the plain mean and population standard
      deviation of the n owned samples (R7); each of `iters` passes keeps the
      owned samples with |y - mu| <= k * sigma (FP64: (double)y - mu, its
      absolute value, k * sigma) and recomputes mu, sigma from the exact
      integer count, sum and sum of squares of the kept samples (sigma from
      the exact numerator n*S2 - S1^2 as in R7). A pass that keeps no sample
      leaves mu, sigma as they were.
  Q2  Median/MAD: mu = lower median of the owned samples, sigma =
      1.4826 * lower median of |y - mu| (integers, so both are exact).
  Q3  Either replaces (mu, sigma) of R7 in S/N = (B - w*mu)/(sigma*sqrt(w));
      sigma == 0 still means no candidates. The boxcar sums, cells, ties and
      threshold are unchanged.
  Q4  De-reddening by running-median subtraction (Section 3.3), with the
      median window moved in strides of a block of D samples (D = 1 would be
      the per-sample running median): block k of the series (samples
      [kD, kD + D) of its L = N_r + w_max - 1 columns) gets
      base_k = lower median of the samples in blocks k - h .. k + h (clipped
      to the series; window (2h + 1) D, which the paper wants above twice the
      widest pulse), and the searched series is
      y''[j] = clip(y[j] - base_{j // D} + M // 2, 0, M), M = nchan * 255 * dec
      the plane's full scale: re-centred at half scale so it stays a
      non-negative integer within every bound of the plain plane (the clip
      only acts on samples more than M / 2 from their baseline; the constant
      moves mu and leaves sigma and the S/N alone). The moments, the noise
      estimate and the boxcar sums are all taken on y''.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

__all__ = ["clipped_moments", "median_mad", "robust_mean_sigma", "block_baseline",
           "dereddened"]

MAD_SCALE = 1.4826


def _mean_sigma(n: int, s1: int, s2: int) -> Tuple[float, float]:
    mu = float(s1) / float(n)
    d = n * s2 - s1 * s1
    return mu, (math.sqrt(float(d)) / float(n)) if d > 0 else 0.0


def clipped_moments(y: np.ndarray, n: int, k: float, iters: int):
    """(count, S1, S2, mu, sigma) after `iters` clipping passes (Q1)."""
    v = y[:n].astype(np.int64)
    cnt, s1, s2 = n, int(v.sum()), int((v * v).sum())
    mu, sigma = _mean_sigma(cnt, s1, s2)
    for _ in range(iters):
        keep = np.abs(v.astype(np.float64) - mu) <= k * sigma
        c = int(keep.sum())
        if c == 0:
            break
        kv = v[keep]
        cnt, s1, s2 = c, int(kv.sum()), int((kv * kv).sum())
        mu, sigma = _mean_sigma(cnt, s1, s2)
    return cnt, s1, s2, mu, sigma


def median_mad(y: np.ndarray, n: int) -> Tuple[float, float]:
    """(median, 1.4826 * MAD) with lower medians (Q2)."""
    v = np.sort(y[:n].astype(np.int64))
    med = int(v[(n - 1) // 2])
    dev = np.sort(np.abs(y[:n].astype(np.int64) - med))
    mad = int(dev[(n - 1) // 2])
    return float(med), MAD_SCALE * float(mad)


def robust_mean_sigma(y: np.ndarray, n: int, mode) -> Tuple[float, float]:
    """mode: None (plain, R7), ("clip", k, iters) or ("mad",)."""
    if mode is None:
        v = y[:n].astype(np.int64)
        return _mean_sigma(n, int(v.sum()), int((v * v).sum()))
    if mode[0] == "clip":
        return clipped_moments(y, n, float(mode[1]), int(mode[2]))[3:]
    if mode[0] == "mad":
        return median_mad(y, n)
    raise ValueError(f"unknown statistics mode {mode!r}")


def block_baseline(y: np.ndarray, L: int, D: int, h: int) -> np.ndarray:
    """base_k for every block of the series y[0:L] (Q4)."""
    nb = (L + D - 1) // D
    v = y[:L].astype(np.int64)
    out = np.empty(nb, dtype=np.int64)
    for k in range(nb):
        w = np.sort(v[max(0, (k - h) * D):min(L, (k + h + 1) * D)])
        out[k] = w[(len(w) - 1) // 2]
    return out


def dereddened(y: np.ndarray, L: int, D: int, h: int, M: int) -> np.ndarray:
    """y''[j] = clip(y[j] - base_{j // D} + M // 2, 0, M) for j < L (Q4)."""
    base = block_baseline(y, L, D, h)
    j = np.arange(L)
    return np.clip(y[:L].astype(np.int64) - base[j // D] + M // 2, 0, M)

