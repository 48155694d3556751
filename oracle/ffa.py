"""Fast Folding Algorithm (FFA) of a dedispersed series and the boxcar search
of its folded profiles (Section 3.5): the series is stacked as m rows of the
base period p, the folding transform turns the stack into m folded profiles
at the linearly spaced trial frequencies of Section 3.5, and a boxcar filter
finds the most significant pulse in each profile. The FFA is Staelin's
(1969) recursion; the split of a stack whose height is not a power of two
follows the head/tail reading below.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper gives the stack, m and the trial frequencies and
periods; the recursion and the profile statistics are not spelled out):
  F1  Series y[0:N) of integers, base period p (integer samples), m =
      floor(N / p) rows, row i = y[i p : i p + p); the samples past m p are
      not folded.
  F2  Folding transform T of a stack of m rows. m = 1: the row itself.
      Otherwise head h = floor(m / 2) rows, tail t = m - h rows, H = T(head),
      U = T(tail), and for s = 0 .. m-1
        k_h = round(s (h - 1) / (m - 1)),  k_t = round(s (t - 1) / (m - 1)),
        sigma = s - k_t,
        T[s][j] = H[k_h][j] + U[k_t][(j + sigma) mod p],
      round(x) = floor(x + 1/2) taken exactly on the integer ratio. Profile s
      drifts s bins over the m - 1 row steps (its last row is shifted by
      exactly s, its first by 0); for m a power of two k_h = k_t = s // 2 and
      this is the classic FFA. Sums are exact integers.
  F3  Trial frequency and period of profile s as the paper gives them:
      f_s = (1/p - s / ((m - 1) p^2)) / tau0, p_s = p^2 / (p - s/(m - 1)) tau0
      (m = 1: the single trial p tau0).
  F4  Noise: mu, sigma = mean and population standard deviation of the m p
      folded samples from their exact integer sums (as the search's moments);
      a folded bin of noise then has mean m mu and deviation sqrt(m) sigma.
  F5  Circular boxcar B_w[s][j] = sum over k < w of T[s][(j + k) mod p] for
      each width w (1 <= w < p), S/N = (B - w m mu) / (sigma sqrt(m w)) in
      FP64; sigma = 0 gives S/N 0 everywhere.
  F6  Best of profile s: the largest S/N, ties to the smaller bin j, then the
      smaller width (the search's order); with sigma = 0 it is (0, 0, w_1).
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

__all__ = ["stack_rows", "round_ratio", "ffa_transform", "trial_periods", "trial_frequencies",
           "fold_moments", "circular_boxcar_sums", "profile_snr", "ffa_search"]


def stack_rows(y: np.ndarray, p: int) -> np.ndarray:
    """m x p stack of the series (F1), int64."""
    m = len(y) // p
    if p < 1 or m < 1:
        raise ValueError("need p >= 1 and at least one full row")
    return np.asarray(y[:m * p], dtype=np.int64).reshape(m, p)


def round_ratio(a: int, b: int) -> int:
    """floor(a / b + 1/2) for integers a >= 0, b > 0 (F2)."""
    return (2 * a + b) // (2 * b)


def ffa_transform(rows: np.ndarray) -> np.ndarray:
    """Folding transform of an m x p integer stack (F2)."""
    m, p = rows.shape
    if m == 1:
        return rows.copy()
    h = m // 2
    t = m - h
    H = ffa_transform(rows[:h])
    U = ffa_transform(rows[h:])
    out = np.empty_like(rows)
    for s in range(m):
        kh = round_ratio(s * (h - 1), m - 1)
        kt = round_ratio(s * (t - 1), m - 1)
        sig = s - kt
        out[s] = H[kh] + np.roll(U[kt], -sig)
    return out


def trial_frequencies(p: int, m: int, tau0: float) -> np.ndarray:
    """f_s of every profile (F3)."""
    if m == 1:
        return np.array([1.0 / (p * tau0)])
    s = np.arange(m, dtype=np.float64)
    return (1.0 / p - s / ((m - 1) * p * p)) / tau0


def trial_periods(p: int, m: int, tau0: float) -> np.ndarray:
    """p_s of every profile (F3)."""
    if m == 1:
        return np.array([p * tau0])
    s = np.arange(m, dtype=np.float64)
    return p * p / (p - s / (m - 1)) * tau0


def fold_moments(y: np.ndarray, p: int) -> Tuple[int, int, int, float, float]:
    """(n, S1, S2, mu, sigma) of the m p folded samples (F4)."""
    v = stack_rows(y, p).ravel().astype(object)  # Python integers: no overflow
    n = int(v.size)
    s1 = int(v.sum())
    s2 = int((v * v).sum())
    mu = float(s1) / float(n)
    d = n * s2 - s1 * s1
    return n, s1, s2, mu, (math.sqrt(float(d)) / float(n)) if d > 0 else 0.0


def circular_boxcar_sums(prof: np.ndarray, w: int) -> np.ndarray:
    """Circular boxcar sums of one profile (F5)."""
    p = len(prof)
    ext = np.concatenate([prof, prof[:w - 1]]).astype(np.int64)
    c = np.concatenate([[0], np.cumsum(ext)])
    return c[w:w + p] - c[:p]


def profile_snr(prof: np.ndarray, widths: Sequence[int], m: int, mu: float, sigma: float):
    """S/N [len(widths)][p] of one folded profile (F5)."""
    out = np.zeros((len(widths), len(prof)))
    if sigma == 0.0:
        return out
    for k, w in enumerate(widths):
        b = circular_boxcar_sums(prof, w).astype(np.float64)
        out[k] = (b - w * m * mu) / (sigma * math.sqrt(m * w))
    return out


def _best(snr: np.ndarray, widths: Sequence[int]) -> Tuple[float, int, int]:
    """F6 order: largest S/N, then smaller j, then smaller width (per width
    the first maximum, then the widths compared in that order)."""
    best = None
    for k, w in enumerate(widths):
        j = int(np.argmax(snr[k]))
        c = (float(snr[k, j]), j, int(w))
        if best is None or c[0] > best[0] or (c[0] == best[0] and (c[1], c[2]) < best[1:]):
            best = c
    return best


def ffa_search(y: np.ndarray, p: int, widths: Sequence[int]):
    """Folded profiles [m][p] (int64), the moments (n, S1, S2, mu, sigma)
    and the best (S/N, bin, width) of every profile (F1-F6)."""
    if any(not (1 <= w < p) for w in widths) or not widths:
        raise ValueError("widths must lie in 1 .. p-1")
    rows = stack_rows(y, p)
    m = rows.shape[0]
    T = ffa_transform(rows)
    mom = fold_moments(y, p)
    mu, sigma = mom[3], mom[4]
    best: List[Tuple[float, int, int]] = []
    for s in range(m):
        if sigma == 0.0:
            best.append((0.0, 0, int(widths[0])))
        else:
            best.append(_best(profile_snr(T[s], widths, m, mu, sigma), widths))
    return T, mom, best
