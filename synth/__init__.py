"""Seeded synthetic GMRT-shaped filterbanks.

This module only makes inputs: 8-bit noise, pulses added at caller-given
per-channel sample offsets, and the parameter sets of the standard workloads.
It holds none of the dedispersion or search arithmetic. Wherever a pulse must
follow a dispersion sweep, the caller passes the per-channel delays in (the
tests take them from the oracle, the benchmark from the library's plan).

Stand-ins: the paper's data (uGMRT pulsar observations and live SPOTLIGHT
beams, Sections 2.4 and 3.2) is not available, so every input is synthetic:
8-bit samples (Section 2.4), 4096 channels stored as spectra (Section 2.2),
noise of a given mean and standard deviation, plus injected dispersed pulses
(the injection-testing method of Section 2.4).

Noise recipe: x = clip(rint(N(mean, std)), 0, 255) drawn through an inverse-CDF
table of 65536 equiprobable cells (so a uint16 uniform draw maps to one uint8
value). Random streams: numpy PCG64 seeded by SeedSequence([seed, *ids]); the
rows are drawn channel by channel in ascending order, so a result depends only
on the seed, the ids and the shape.
"""
from __future__ import annotations

import dataclasses
from statistics import NormalDist
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "candidate_list",
    "normal_u8_table", "filterbank", "inject_pulse", "to_time_major",
    "Pulse", "Workload", "tiny", "full_band", "multi_range", "batched_beams",
    "stream_beam_params",
]

_TABLE_BITS = 16


def normal_u8_table(mean: float, std: float) -> np.ndarray:
    """uint8[65536]: cell u holds clip(rint(q), 0, 255) with q the
    (u + 0.5)/65536 quantile of N(mean, std)."""
    nd = NormalDist(mean, std)
    n = 1 << _TABLE_BITS
    q = np.array([nd.inv_cdf((u + 0.5) / n) for u in range(n)], dtype=np.float64)
    return np.clip(np.rint(q), 0, 255).astype(np.uint8)


_TABLE_CACHE: dict = {}


def _table(mean: float, std: float) -> np.ndarray:
    key = (float(mean), float(std))
    t = _TABLE_CACHE.get(key)
    if t is None:
        t = normal_u8_table(mean, std)
        _TABLE_CACHE[key] = t
    return t


def filterbank(seed: int, nchan: int, nsamp: int, mean: float = 128.0,
               std: float = 16.0, ids: Sequence[int] = ()) -> np.ndarray:
    """Channel-major uint8 noise filterbank x[c][t], shape (nchan, nsamp)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, *ids])))
    tab = _table(mean, std)
    out = np.empty((nchan, nsamp), dtype=np.uint8)
    for c in range(nchan):
        u = rng.integers(0, 1 << _TABLE_BITS, size=nsamp, dtype=np.uint16)
        np.take(tab, u, out=out[c])
    return out


def inject_pulse(x: np.ndarray, offsets: np.ndarray, t0: int, width: int,
                 amp: float, seed: int = 0) -> int:
    """Add a top-hat pulse in place: x[c][t0 + offsets[c] + k] gains amp
    counts for k < width, saturating at 255. A whole amp is added exactly; a
    fractional amp is dithered (floor(amp) plus one with probability
    frac(amp), from a stream seeded by (seed, t0, width)), so the expected
    increment is amp. Samples outside the array are skipped. Returns the
    number of saturated samples."""
    base = int(np.floor(amp))
    frac = float(amp) - base
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, t0, width, 99])))
    nchan, nsamp = x.shape
    clipped = 0
    for c in range(nchan):
        a = int(t0 + offsets[c])
        lo, hi = max(a, 0), min(a + width, nsamp)
        if lo >= hi:
            continue
        inc = np.full(hi - lo, base, dtype=np.int32)
        if frac > 0.0:
            inc += (rng.random(hi - lo) < frac).astype(np.int32)
        seg = x[c, lo:hi].astype(np.int32) + inc
        clipped += int(np.count_nonzero(seg > 255))
        x[c, lo:hi] = np.clip(seg, 0, 255).astype(np.uint8)
    return clipped


def to_time_major(x: np.ndarray) -> np.ndarray:
    """Spectra layout [t][c] (how the beamformer writes its blocks)."""
    return np.ascontiguousarray(x.T)


@dataclasses.dataclass
class Pulse:
    dm: float
    t0: int          # arrival sample at the highest-frequency channel
    width: int       # samples
    amp: float       # counts added per channel per sample


@dataclasses.dataclass
class Workload:
    """One input set plus the search parameters it is run with.

    Exactly one of dm_list / ranges is set. ranges are (lo, hi, step, dec)."""
    name: str
    freqs_mhz: np.ndarray
    t_samp: float
    dm_list: Optional[np.ndarray]
    ranges: Optional[List[Tuple[float, float, float, int]]]
    widths: List[int]
    cand_block: int
    threshold: float
    x: Optional[np.ndarray]          # channel-major uint8 [C][T]
    pulses: List[Pulse]
    nsamp: int = 0

    @property
    def nchan(self) -> int:
        return len(self.freqs_mhz)


DelayFn = Callable[[np.ndarray, np.ndarray, float], np.ndarray]
"""delay_fn(freqs_mhz, dms, t_samp) -> int array [len(dms)][nchan] of
per-channel sample delays at decimation 1."""


def _inject_all(x, pulses, freqs, t_samp, delay_fn: DelayFn) -> None:
    if not pulses:
        return
    d = delay_fn(freqs, np.array([p.dm for p in pulses], dtype=np.float64), t_samp)
    for k, p in enumerate(pulses):
        inject_pulse(x, d[k], p.t0, p.width, p.amp)


def tiny(delay_fn: DelayFn, seed: int = 1, with_data: bool = True) -> Workload:
    """256 channels 500 -> 300 MHz (top first), 1.31072 ms, 8192 samples,
    N(128,16); one pulse at DM 100, arrival sample 3000 at the top channel,
    width 4, +40 counts; DM trials 0..200 step 1; widths 1,2,4,8,16."""
    freqs = np.linspace(500.0, 300.0, 256)
    t_samp = 1.31072e-3
    T = 8192
    pulses = [Pulse(100.0, 3000, 4, 40.0)]
    x = None
    if with_data:
        x = filterbank(seed, 256, T, 128.0, 16.0)
        _inject_all(x, pulses, freqs, t_samp, delay_fn)
    return Workload("tiny-256ch-201dm-8192", freqs, t_samp,
                    np.arange(201, dtype=np.float64), None, [1, 2, 4, 8, 16],
                    1024, 7.0, x, pulses, T)


def _random_pulses(rng, n, dm_lo, dm_hi, n_owned, nchan, std):
    out = []
    for _ in range(n):
        dm = float(rng.uniform(dm_lo, dm_hi))
        w = int(np.rint(2.0 ** rng.uniform(0.0, 6.0)))
        snr = float(rng.uniform(5.0, 30.0))
        t0 = int(rng.integers(0, max(1, n_owned - w)))
        out.append(Pulse(dm, t0, w, snr * std / np.sqrt(nchan * w)))
    return out


def full_band(delay_fn: DelayFn, seed: int = 2, n_owned: int = 1 << 18,
              nchan: int = 4096, ndm: int = 2048, dm_max: float = 1000.0,
              widths: Sequence[int] = (), with_data: bool = True) -> Workload:
    """4096 channels 750 -> 550 MHz, 81.92 us, n_owned samples plus the
    max-delay overlap, N(128,16), 20 pulses at DM U[50,1000], widths 1-64,
    matched S/N 5-30; ndm uniform DM trials over [0, dm_max] inclusive."""
    freqs = np.linspace(750.0, 550.0, nchan)
    t_samp = 81.92e-6
    dms = np.linspace(0.0, dm_max, ndm)
    overlap = int(np.max(delay_fn(freqs, dms[-1:], t_samp)))
    if widths:
        overlap += max(widths) - 1
    T = n_owned + overlap
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7777])))
    pulses = _random_pulses(rng, 20, 50.0, min(1000.0, dm_max), n_owned, nchan, 16.0)
    x = None
    if with_data:
        x = filterbank(seed, nchan, T, 128.0, 16.0)
        _inject_all(x, pulses, freqs, t_samp, delay_fn)
    return Workload(f"full-band-{nchan}ch-{ndm}dm-{n_owned}", freqs, t_samp, dms,
                    None, list(widths), 1024, 7.0, x, pulses, T)


MULTI_RANGES = [(0.0, 100.0, 0.1, 1), (100.0, 300.0, 0.2, 2), (300.0, 700.0, 0.5, 4),
                (700.0, 1500.0, 1.0, 8), (1500.0, 3000.0, 2.0, 16)]


def multi_range(overlap: int, seed: int = 3, n_owned: int = 1 << 19,
                nchan: int = 4096, ranges=None, widths=None,
                delay_fn: Optional[DelayFn] = None, with_data: bool = True) -> Workload:
    """4096 channels 750 -> 550 MHz, 81.92 us, n_owned + overlap samples;
    five DM ranges with decimation 1..16; widths 1..256 (powers of two);
    threshold 7. overlap comes from the plan (it depends on the delays)."""
    freqs = np.linspace(750.0, 550.0, nchan)
    t_samp = 81.92e-6
    ranges = list(ranges or MULTI_RANGES)
    widths = list(widths or [1 << k for k in range(9)])
    T = n_owned + overlap
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7777])))
    pulses = _random_pulses(rng, 20, 50.0, 2900.0, n_owned, nchan, 16.0)
    x = None
    if with_data:
        x = filterbank(seed, nchan, T, 128.0, 16.0)
        if delay_fn is not None:
            _inject_all(x, pulses, freqs, t_samp, delay_fn)
    return Workload(f"multi-range-{nchan}ch-{n_owned}", freqs, t_samp, None, ranges,
                    widths, 1024, 7.0, x, pulses, T)


def batched_beams(seed: int = 4, nbeams: int = 32, lo: int = 1 << 16, hi: int = 1 << 18):
    """Per-beam (owned length, mean, std) for the many-beam workload:
    lengths U[lo, hi], mean U[100,150], std U[8,24]."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 4444])))
    out = []
    for b in range(nbeams):
        n = int(rng.integers(lo, hi + 1))
        out.append((n, float(rng.uniform(100.0, 150.0)), float(rng.uniform(8.0, 24.0))))
    return out


def stream_beam_params(nbeams: int = 160):
    """Channel count per beam for the streaming workload: beam b gets
    [1024, 2048, 4096][b % 3] channels over 750 -> 550 MHz."""
    return [[1024, 2048, 4096][b % 3] for b in range(nbeams)]


def candidate_list(seed: int, ndm: Sequence[int], n_owned: Sequence[int], n_events: int = 40,
                   per_event: int = 30, n_noise: int = 200, max_width: int = 64):
    """Seeded candidate lists in the search's output order (range, DM index,
    sample) for testing candidate sifting: events (clumps of candidates
    spread over a few trials and samples around a centre, S/N falling away
    from it, quantised to 1/8 so that ties occur) plus scattered weak
    candidates. Returns (range, dm_index, sample, width, snr float32)
    arrays. ndm / n_owned give each range's trial count and owned samples."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 77])))
    nr = len(ndm)
    rows = []
    for _ in range(n_events):
        r = int(g.integers(0, nr))
        ci = int(g.integers(0, ndm[r]))
        cs = int(g.integers(0, n_owned[r]))
        peak = float(g.uniform(8.0, 40.0))
        for _ in range(per_event):
            di = int(round(g.normal(0.0, 3.0)))
            ds = int(round(g.normal(0.0, 40.0)))
            i, s = ci + di, cs + ds
            if 0 <= i < ndm[r] and 0 <= s < n_owned[r]:
                snr = peak - 0.4 * abs(di) - 0.02 * abs(ds) - float(g.exponential(0.5))
                rows.append((r, i, s, int(g.integers(1, max_width + 1)), max(snr, 6.0)))
    for _ in range(n_noise):
        r = int(g.integers(0, nr))
        rows.append((r, int(g.integers(0, ndm[r])), int(g.integers(0, n_owned[r])),
                     int(g.integers(1, max_width + 1)), float(g.uniform(6.0, 9.0))))
    # one candidate per (range, trial, sample), as the search reports at most one
    # per cell; quantised S/N makes ties frequent
    uniq = {}
    for r, i, s, w, snr in rows:
        uniq[(r, i, s)] = (w, np.float32(round(snr * 8.0) / 8.0))
    keys = sorted(uniq)
    rng_ = np.array([k[0] for k in keys], dtype=np.int32)
    dmi = np.array([k[1] for k in keys], dtype=np.int32)
    smp = np.array([k[2] for k in keys], dtype=np.int64)
    wid = np.array([uniq[k][0] for k in keys], dtype=np.int32)
    snr = np.array([uniq[k][1] for k in keys], dtype=np.float32)
    return rng_, dmi, smp, wid, snr

