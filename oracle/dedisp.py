"""FP64 / exact-integer oracle: delays, decimation, brute-force dedispersion,
moments, boxcar S/N, per-DM best and candidates.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of points the paper leaves open (each one is a convention, stated
once here and used by every function below):

  R1  Delay constant K = 4.148808e3 s MHz^2 pc^-1 cm^3 (Chapter 1, Eq. (1)
      prints the same law as 4.14881 ms GHz^2 pc^-1 cm^3, a 6-digit rounding
      of it). DM in pc cm^-3, frequencies in MHz, sampling time in seconds.
  R2  Reference frequency f_top = the highest listed channel frequency, so
      every delay is >= 0 and the top channel has delay 0.
  R3  Sample delay d = floor(v + 0.5) (round half up) with
      v = K * DM * (1/(f*f) - 1/(f_top*f_top)) / (dec * t_samp), evaluated
      left to right in FP64: ((K * DM) * diff) / (float(dec) * t_samp).
  R4  Downsampling (Section 3.2) is applied BEFORE dedispersion, as an exact
      sum of dec consecutive samples (not a mean), groups aligned to sample 0
      of the input; delays and boxcar widths of a range are in its own
      decimated samples.
  R5  Overlap O = max over ranges of (max delay_r + w_max - 1) * dec_r native
      samples (w_max = 1 when no widths are searched). With T input samples,
      N = T - O owned native samples; range r owns N_r = N // dec_r samples
      and its plane has N_r + w_max - 1 columns.
  R6  Boxcar window sums B_w[j] = sum_{k<w} y[j+k] indexed by the window
      start j, for every owned start j < N_r and every width w.
  R7  S/N = (B_w - w*mu) / (sigma*sqrt(w)), mu and sigma the mean and the
      population standard deviation of the owned samples of that DM trial:
      mu = S1/n, sigma = sqrt(n*S2 - S1^2) / n with S1, S2 the exact integer
      sums of y and y^2 and the numerator formed exactly. If n*S2 == S1^2 the
      series is constant: every S/N is 0 and it yields no candidate.
  R8  Ties: the best (j, w) is the first maximum in (j ascending, w ascending)
      order.
  R9  A candidate is the best (S/N, j, w) of one cell of cand_block owned
      starts of one DM trial, kept when S/N > threshold (strict). The list is
      ordered by (range, DM index, sample).
  R10 DM ranges (lo, hi, step, dec): DM_i = lo + i*step in FP64 for
      i < floor((hi - lo)/step + 0.5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "K_DM", "dm_range_values", "delay_table", "decimate", "corner_turn",
    "overlap_samples", "dedisperse", "dedisperse_rows", "row_moments",
    "mean_sigma", "boxcar_sums", "snr_matrix", "best_of", "search_row",
    "PlanSpec", "RangeSpec", "make_plan", "run", "RowResult", "plane_checksums",
]

K_DM = 4.148808e3  # s MHz^2 pc^-1 cm^3 (R1)


def dm_range_values(lo: float, hi: float, step: float) -> np.ndarray:
    """Trial DMs of one range (R10)."""
    count = int(math.floor((hi - lo) / step + 0.5))
    return np.array([lo + i * step for i in range(count)], dtype=np.float64)


def delay_table(freqs_mhz: Sequence[float], dms: Sequence[float], t_samp: float,
                dec: int = 1) -> np.ndarray:
    """Integer channel delays, int64 [ndm][nchan] (Chapter 1, Eq. (1); R1-R3).

    Delay of channel c at trial DM_i, relative to the highest listed frequency,
    in samples of width dec * t_samp, rounded half up."""
    f = np.asarray(freqs_mhz, dtype=np.float64)
    dm = np.asarray(dms, dtype=np.float64)
    f_top = float(np.max(f))
    diff = 1.0 / (f * f) - 1.0 / (f_top * f_top)
    den = float(dec) * float(t_samp)
    v = (K_DM * dm[:, None]) * diff[None, :] / den
    return np.floor(v + 0.5).astype(np.int64)


def decimate(x: np.ndarray, dec: int) -> np.ndarray:
    """Section 3.2 downsampling as an exact sum of dec consecutive samples
    (R4): out[c][j] = sum_{k<dec} x[c][j*dec + k], j < T // dec. int64."""
    x = np.asarray(x)
    if dec == 1:
        return x.astype(np.int64)
    n = x.shape[1] // dec
    # int32 holds any sum of dec <= 2^23 uint8/uint16 values exactly
    return x[:, : n * dec].reshape(x.shape[0], n, dec).sum(axis=2, dtype=np.int32)


def corner_turn(x_time_major: np.ndarray) -> np.ndarray:
    """Spectra [t][c] -> channel rows [c][t]."""
    return np.ascontiguousarray(np.asarray(x_time_major).T)


def overlap_samples(max_delays: Sequence[int], decs: Sequence[int], w_max: int) -> int:
    """R5: native-sample look-ahead a chunk needs beyond its owned samples."""
    return max((int(d) + w_max - 1) * int(r) for d, r in zip(max_delays, decs))


def dedisperse(xr: np.ndarray, delays: np.ndarray, length: int) -> np.ndarray:
    """Brute-force incoherent dedispersion (Section 3.2, Section 2.1):
    y[i][j] = sum_c xr[c][j + delays[i][c]] for j < length. int64."""
    return dedisperse_rows(xr, delays, range(delays.shape[0]), length)


def dedisperse_rows(xr: np.ndarray, delays: np.ndarray, rows, length: int) -> np.ndarray:
    """dedisperse() restricted to the given DM rows (same sum, one row at a time)."""
    xr = np.asarray(xr)  # uint8/int32 rows are added into int64 sums below
    rows = list(rows)
    nchan = xr.shape[0]
    y = np.zeros((len(rows), length), dtype=np.int64)
    for k, i in enumerate(rows):
        for c in range(nchan):
            d = int(delays[i][c])
            y[k] += xr[c, d:d + length]
    return y


def plane_checksums(xr: np.ndarray, delays: np.ndarray, length: int) -> Tuple[np.ndarray,
                                                                             np.ndarray]:
    """Two exact checksums of every row of the dedispersed plane, without
    forming the plane: A[i] = sum_{j<length} y[i][j] and
    B[i] = sum_{j<length} j * y[i][j], y as in dedisperse().

    Each channel contributes the samples [d, d + length) of its row, d its
    delay at trial i, so with per-channel prefix sums P[k] = sum_{t<k} x[t]
    and Q[k] = sum_{t<k} t * x[t]:
      A[i] = sum_c P[d + length] - P[d]
      B[i] = sum_c (Q[d + length] - Q[d]) - d * (P[d + length] - P[d]).
    int64 (exact while B stays below 2^63). Channels are taken one at a time
    so memory stays at a few rows."""
    xr = np.asarray(xr)
    d = np.asarray(delays, dtype=np.int64)
    ndm, nchan = d.shape
    a = np.zeros(ndm, dtype=np.int64)
    b = np.zeros(ndm, dtype=np.int64)
    t = np.arange(xr.shape[1], dtype=np.int64)
    for c in range(nchan):
        row = xr[c].astype(np.int64)
        p = np.concatenate(([0], np.cumsum(row)))
        q = np.concatenate(([0], np.cumsum(row * t)))
        lo, hi = d[:, c], d[:, c] + length
        ps = p[hi] - p[lo]
        a += ps
        b += (q[hi] - q[lo]) - lo * ps
    return a, b


def row_moments(y: np.ndarray, n: int) -> Tuple[int, int]:
    """Exact S1 = sum y[:n], S2 = sum y[:n]^2 (R7), as Python ints."""
    v = np.asarray(y[:n]).astype(np.uint64)
    s1 = int(np.sum(v, dtype=np.uint64))
    s2 = int(np.sum(v * v, dtype=np.uint64))
    # the uint64 sums are exact when no wrap happened; confirm with Python ints
    # on small rows (cheap) so a silent wrap can never pass
    if n <= 4096:
        assert s2 == sum(int(a) * int(a) for a in np.asarray(y[:n]).tolist())
    return s1, s2


def mean_sigma(s1: int, s2: int, n: int) -> Tuple[float, float]:
    """R7: mu = S1/n; sigma = sqrt(n*S2 - S1^2)/n (0 for a constant series)."""
    mu = float(s1) / float(n)
    d = n * s2 - s1 * s1
    if d < 0:
        raise ValueError("moments inconsistent")
    sigma = math.sqrt(float(d)) / float(n) if d > 0 else 0.0
    return mu, sigma


def boxcar_sums(y: np.ndarray, w: int, n: int) -> np.ndarray:
    """R6: B_w[j] = sum_{k<w} y[j+k] for j < n (time-domain boxcar filter,
    Section 2.1). int64."""
    y = np.asarray(y).astype(np.int64)
    if len(y) < n + w - 1:
        raise ValueError("row too short for the boxcar look-ahead")
    b = np.zeros(n, dtype=np.int64)
    for k in range(w):
        b += y[k:k + n]
    return b


def snr_matrix(y: np.ndarray, widths: Sequence[int], n: int, mu: float,
               sigma: float) -> np.ndarray:
    """FP64 S/N for every owned start and width, shape [n][len(widths)] (R7)."""
    out = np.zeros((n, len(widths)), dtype=np.float64)
    if sigma == 0.0:
        return out
    for k, w in enumerate(widths):
        b = boxcar_sums(y, w, n).astype(np.float64)
        out[:, k] = (b - float(w) * mu) / (sigma * math.sqrt(float(w)))
    return out


def best_of(snr: np.ndarray, j0: int = 0) -> Tuple[float, int, int]:
    """First maximum in (j, w) order (R8): (S/N, j0 + j, width index)."""
    flat = int(np.argmax(snr.reshape(-1)))
    nw = snr.shape[1]
    j, k = divmod(flat, nw)
    return float(snr[j, k]), j0 + j, k


@dataclass
class RowResult:
    n: int
    s1: int
    s2: int
    mean: float
    std: float
    best: Tuple[float, int, int]          # (S/N fp64, sample j, width)
    cells: List[Tuple[float, int, int]]   # per cell (S/N fp64, j, width)
    cands: List[Tuple[float, int, int]]   # cells with S/N > threshold


def search_row(y: np.ndarray, widths: Sequence[int], n: int, cand_block: int,
               threshold: float, stats=None, dered=None) -> RowResult:
    """Single-pulse search of one dedispersed series (Section 2.1; R6-R9).
    stats selects the noise estimate of the S/N (oracle.robust): None for
    R7's moments, ("clip", k, iters) or ("mad",). s1, s2 are always the
    plain moments of the owned samples of the searched series. dered = (D, h, M) searches the
    de-reddened series instead (oracle.robust, Q4; M the full scale)."""
    if dered is not None:
        from .robust import dereddened
        y = dereddened(y, n + max(widths) - 1, dered[0], dered[1], dered[2])
    s1, s2 = row_moments(y, n)
    if stats is None:
        mu, sigma = mean_sigma(s1, s2, n)
    else:
        from .robust import robust_mean_sigma
        mu, sigma = robust_mean_sigma(y, n, stats)
    snr = snr_matrix(y, widths, n, mu, sigma)
    bs, bj, bk = best_of(snr)
    cells, cands = [], []
    for j0 in range(0, n, cand_block):
        cs, cj, ck = best_of(snr[j0:min(j0 + cand_block, n)], j0)
        cells.append((cs, cj, int(widths[ck])))
        if sigma > 0.0 and cs > threshold:
            cands.append((cs, cj, int(widths[ck])))
    return RowResult(n, s1, s2, mu, sigma, (bs, bj, int(widths[bk])), cells, cands)


@dataclass
class RangeSpec:
    dec: int
    dms: np.ndarray
    delays: np.ndarray   # int64 [ndm][nchan], in decimated samples

    @property
    def max_delay(self) -> int:
        return int(self.delays.max()) if self.delays.size else 0


@dataclass
class PlanSpec:
    freqs_mhz: np.ndarray
    t_samp: float
    ranges: List[RangeSpec]
    widths: List[int]
    cand_block: int
    threshold: float
    stats: Optional[tuple] = None   # noise estimate of the S/N (oracle.robust)
    dered: Optional[tuple] = None   # (D, h) de-reddening of the searched series

    @property
    def w_max(self) -> int:
        return max(self.widths) if self.widths else 1

    @property
    def overlap(self) -> int:
        return overlap_samples([r.max_delay for r in self.ranges],
                               [r.dec for r in self.ranges], self.w_max)

    def owned(self, nsamp_in: int) -> List[int]:
        """N_r per range (R5); raises if the input is shorter than O + 1."""
        n = nsamp_in - self.overlap
        if n < 1:
            raise ValueError("input shorter than overlap + 1")
        out = [n // r.dec for r in self.ranges]
        if min(out) < 1:
            raise ValueError("a decimated range owns no sample")
        return out


def make_plan(freqs_mhz, t_samp, dm_list=None, ranges=None, widths=(),
              cand_block=1024, threshold=7.0, stats=None, dered=None) -> PlanSpec:
    """Plan from an explicit DM list (decimation 1) or from DM ranges
    (lo, hi, step, dec)."""
    if (dm_list is None) == (ranges is None):
        raise ValueError("give exactly one of dm_list / ranges")
    specs = []
    if dm_list is not None:
        dms = np.asarray(dm_list, dtype=np.float64)
        specs.append(RangeSpec(1, dms, delay_table(freqs_mhz, dms, t_samp, 1)))
    else:
        for lo, hi, step, dec in ranges:
            dms = dm_range_values(lo, hi, step)
            specs.append(RangeSpec(int(dec), dms, delay_table(freqs_mhz, dms, t_samp, int(dec))))
    return PlanSpec(np.asarray(freqs_mhz, dtype=np.float64), float(t_samp), specs,
                    list(widths), int(cand_block), float(threshold), stats,
                    None if dered is None else (int(dered[0]), int(dered[1])))


def run(plan: PlanSpec, x: np.ndarray, rows: Optional[List[Sequence[int]]] = None,
        search: bool = True):
    """Whole path on a channel-major input x[c][t].

    Returns, per range, (row indices, plane rows int64 [len(rows)][N_r+w_max-1],
    RowResult list or None). rows[r] restricts range r to some DM rows."""
    owned = plan.owned(x.shape[1])
    out = []
    for r, spec in enumerate(plan.ranges):
        xr = x if spec.dec == 1 else decimate(x, spec.dec)
        length = owned[r] + plan.w_max - 1
        rr = list(range(len(spec.dms))) if rows is None else list(rows[r])
        y = dedisperse_rows(xr, spec.delays, rr, length)
        res = None
        if search and plan.widths:
            dr = None
            if plan.dered is not None:
                dr = (plan.dered[0], plan.dered[1], len(plan.freqs_mhz) * 255 * spec.dec)
            res = [search_row(y[k], plan.widths, owned[r], plan.cand_block, plan.threshold,
                              plan.stats, dr)
                   for k in range(len(rr))]
        out.append((rr, y, res))
    return out
