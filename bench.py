#!/usr/bin/env python3
"""Throughput benchmark of the hot path on one MI355X.

One step = one pass of the whole path over one chunk of the full-band beam:
corner turn of the spectra-ordered uint8 input, brute-force dedispersion over
2048 trial DMs (0-1000 pc cm^-3) of 4096 channels (750 -> 550 MHz, 81.92 us)
for 2^18 owned samples plus the max-delay overlap, then the boxcar
single-pulse search (widths 1..64) with exact moments, S/N and candidate
compaction. Inputs are synthetic (seeded GMRT-shaped noise plus injected
dispersed pulses) and resident in HBM before the timed region.

Prints one JSON line. Metric: Gchan.DM.samples/s = nchan * ndm * N_owned /
time. The dedispersion kernel's own duration comes from HIP events the
library records on the launch stream.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dedispersion Gchan·DM·samples/s; real-time beams served + p99 chunk latency"
UNIT = "Gchan·DM·samples/s"
WIDTHS = [1, 2, 4, 8, 16, 32, 64]
# Vector form of the dedispersion kernel (tile kind 1): MI355X's 256 CUs x 64
# lanes x 2.4 GHz, two integer adds per lane per clock (v_add3_u32)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 * 2 / 1e12
# Matrix-core form (tile kind 5): one v_mfma_i32_16x16x64_i8 (16384 int8 MACs,
# 32768 ops) adds two channels into 256 samples of one trial, 512 adds: 64
# MFMA ops per add, so the dense int8 MFMA peak of 5.0 POP/s is 78.1 T adds/s
MFMA_OPS_PER_ADD = 64
MFMA_PEAK_POPS = 5.0
MFMA_PEAK_TOPS = MFMA_PEAK_POPS * 1e3 / MFMA_OPS_PER_ADD
# LDS bytes per add of each form's interior stage, per wavefront:
#   vector, tile [1, 2, 8, 1, 8, 8]: 32 64-bit + 32 32-bit reads and at most 4
#   128-bit staging stores for 16384 adds (8 channels x 2 trials x 1024 samples);
#   matrix core, tile [5, 1, 16, 1, 16, 16]: 8 (pair, trial) groups of one
#   selection-table read and 8 data reads (128-bit each) and at most 3 128-bit
#   staging stores for 32768 adds (16 channels x 1 trial x 2048 samples);
#   tile [5, 2, 8, 1, 8, 16]: 16 groups of one table read and 4 data reads and
#   at most 4 staging stores for 32768 adds (16 channels x 2 trials x 1024)
# against the LDS rate of ds_read_b128 (237 B per clock per CU stored; the
# ceiling probe's own measurement replaces it when the probe runs)
LDS_BYTES_PER_ADD = {(1, 2, 8, 1, 8, 8): (32 * 512 + 32 * 256 + 4 * 1024) / 16384,
                     (5, 1, 16, 1, 16, 16): (8 * 9 * 1024 + 3 * 1024) / 32768,
                     (5, 2, 8, 1, 8, 16): (16 * 5 * 1024 + 4 * 1024) / 32768}
LDS_PEAK_TBPS = 237 * 256 * 2.4e9 / 1e12
# HBM bytes of one dedispersion launch of this workload, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE scaled by a copy kernel of known size (profiles/k_dedisp_vector_full_band_hbm_bytes.md,
# profiles/k_dedisp_mfma_full_band_hbm_bytes.md).
# Valid for the tile shape it was taken with; any other shape reports null.
MEASURED_TRAFFIC = {(1, 2, 8, 1, 8, 8): 61.13e9, (5, 2, 8, 1, 8, 16): 52.34e9,
                    (5, 1, 16, 1, 16, 16): 29.75e9}
# Adds per VALU instruction of the vector form for that tile, from the SQ
# counters (profiles/k_dedisp_vector_full_band_sq_counters.md)
ADDS_PER_VALU = {(1, 2, 8, 1, 8, 8): 66.3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def _oracle_rows(w, d, sel, cols, n_owned, threads: int) -> float:
    """Wall seconds for the oracle (dedispersion + boxcar search) of the DM
    rows `sel`, shared among `threads` host threads (numpy releases the GIL
    in the row additions)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle

    def one(k):
        y = oracle.dedisperse(w.x, d[k:k + 1], cols)
        oracle.search_row(y[0], WIDTHS, n_owned, 1024, 7.0)

    t0 = time.perf_counter()
    if threads == 1:
        for k in range(len(sel)):
            one(k)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(len(sel))))
    return time.perf_counter() - t0


def host_threads() -> int:
    """Host threads for the oracle's all-core timing: the CPU share of one
    GPU on the box (at most 16), or fewer if the host has fewer."""
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(w, plan_delays, rows: int):
    """The oracle as it stands, on a bounded sample of DM trials of the same
    input and owned length (dedispersion + search), timed on one host thread
    (as the paper's single-thread CPU baseline) and on all of the host's
    threads; plus the tiny workload timed in full."""
    import oracle
    import synth
    n_owned = w.nsamp - (int(plan_delays.max()) + max(WIDTHS) - 1)
    cols = n_owned + max(WIDTHS) - 1
    nth = host_threads()
    sel1 = np.linspace(0, len(w.dm_list) - 1, rows).astype(int)
    d1 = oracle.delay_table(w.freqs_mhz, w.dm_list[sel1], w.t_samp)
    dt1 = _oracle_rows(w, d1, sel1, cols, n_owned, 1)
    seln = np.linspace(0, len(w.dm_list) - 1, rows * max(1, nth // 2)).astype(int)
    dn = oracle.delay_table(w.freqs_mhz, w.dm_list[seln], w.t_samp)
    dtn = _oracle_rows(w, dn, seln, cols, n_owned, nth)
    v1 = w.nchan * len(sel1) * n_owned / dt1 / 1e9
    vn = w.nchan * len(seln) * n_owned / dtn / 1e9
    # the tiny workload (256 channels, 201 trials, 8192 samples), in full
    t = synth.tiny(oracle.delay_table)
    spec = oracle.make_plan(t.freqs_mhz, t.t_samp, dm_list=t.dm_list, widths=t.widths,
                            cand_block=t.cand_block, threshold=t.threshold)
    t0 = time.perf_counter()
    oracle.run(spec, t.x)
    dtt = time.perf_counter() - t0
    n_t = spec.owned(t.nsamp)[0]
    model = cpu_model()
    return {"value": round(v1, 4), "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"{len(sel1)} of {len(w.dm_list)} DM trials (evenly spaced), full 4096 "
                      f"channels x {n_owned} owned samples, dedispersion + boxcar search, numpy "
                      f"FP64/int64 oracle, {dt1:.1f} s on 1 thread of {model} "
                      f"({os.cpu_count()} logical CPUs); the metric is linear in the trials",
            "all_cores": {"value": round(vn, 4), "unit": UNIT, "cores": nth,
                          "sample": f"{len(seln)} DM trials shared among {nth} host threads, "
                                    f"{dtn:.1f} s"},
            "tiny_full": {"value": round(256 * 201 * n_t / dtt / 1e9, 4), "unit": UNIT,
                          "cores": 1, "seconds": round(dtt, 3),
                          "sample": "tiny workload in full: 256 channels x 201 trials x "
                                    f"{n_t} samples, dedispersion + search of every trial"}}


# Candidate sifting measured after the step: stencils of (1, 4) DM steps x (16, 128) samples,
# then clustering with a (10 DM steps, 512 samples) neighbourhood and 2 points per core.
SIFT_STENCILS_STEPS = [(1.0, 16), (4.0, 128)]
SIFT_EPS_STEPS = (10.0, 512)
SIFT_MIN_PTS = 2


def sift_bench(sdd, torch, plan, out, dm_step: float, large: int):
    """Time sdd_sift_candidates (HIP events on its stream) on the step's own
    candidate list and on a seeded list of `large` candidates."""
    import ctypes as C
    import synth
    from paper_2605_03531_amd import _capi as A
    L = A.lib()
    st = [(a * dm_step, b) for a, b in SIFT_STENCILS_STEPS]
    eps = (SIFT_EPS_STEPS[0] * dm_step, SIFT_EPS_STEPS[1])

    def timed(o, reps):
        plan.sift(o, stencils=st, eps=eps, min_pts=SIFT_MIN_PTS)  # warm-up, workspace sizing
        torch.cuda.synchronize()
        A.check(L.sdd_profile_enable(1), "profile")
        for _ in range(reps):
            res = plan.sift(o, stencils=st, eps=eps, min_pts=SIFT_MIN_PTS)
        torch.cuda.synchronize()
        ms, n = C.c_double(), C.c_int64()
        A.check(L.sdd_profile_read(A.STAGES["sift"], C.byref(ms), C.byref(n)), "profile_read")
        L.sdd_profile_enable(0)
        kept, _ = res.host()
        return ms.value / max(n.value, 1), len(kept)

    n_step = min(int(out.ncand.cpu()[0]), out.cands.numel() // sdd.CAND_DTYPE.itemsize)
    ms_step, kept_step = timed(out, 5)
    ndm = plan.ndm_total
    rng, dmi, smp, wid, snr = synth.candidate_list(21, [ndm], [1 << 18], n_events=large // 40,
                                                   per_event=40, n_noise=large // 4)
    rng, dmi, smp, wid, snr = rng[:large], dmi[:large], smp[:large], wid[:large], snr[:large]
    arr = np.zeros(large, dtype=sdd.CAND_DTYPE)
    m = len(rng)
    arr["range"][:m], arr["dm_index"][:m], arr["sample"][:m] = rng, dmi, smp
    arr["width"][:m], arr["snr"][:m] = wid, snr
    big = sdd.SearchOut(None, None, torch.from_numpy(arr.view(np.uint8).copy()).to("cuda:0"),
                        torch.tensor([m], dtype=torch.int32, device="cuda:0"))
    ms_big, kept_big = timed(big, 3)
    return {"stencils": [list(x) for x in st], "eps": list(eps), "min_pts": SIFT_MIN_PTS,
            "step": {"candidates": n_step, "kept": kept_step, "ms": round(ms_step, 4)},
            "seeded_list": {"candidates": m, "kept": kept_big, "ms": round(ms_big, 4)}}


def rfi_bench(sdd, torch, plan, xt, planes, out, ws_unused, reps: int = 3):
    """Time the RFI estimator on the step's chunk and the pre-conditioned step
    (maps applied in the corner turn), both with HIP events on one stream."""
    import ctypes as C
    from paper_2605_03531_amd import _capi as A
    L = A.lib()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        lut, mask, flags = plan.rfi_estimate(xt, stream=s)          # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            lut, mask, flags = plan.rfi_estimate(xt, stream=s)
        e1.record(s)
        e1.synchronize()
        est_ms = e0.elapsed_time(e1) / reps
        plan.dedisperse_search(xt, planes=planes, out=out, lut=lut, time_mask=mask, stream=s)
        s.synchronize()
        A.check(L.sdd_profile_enable(1), "profile")
        e0.record(s)
        for _ in range(reps):
            plan.dedisperse_search(xt, planes=planes, out=out, lut=lut, time_mask=mask, stream=s)
        e1.record(s)
        e1.synchronize()
        step_ms = e0.elapsed_time(e1) / reps
        ms, n = C.c_double(), C.c_int64()
        A.check(L.sdd_profile_read(A.STAGES["corner_turn"], C.byref(ms), C.byref(n)), "read")
        L.sdd_profile_enable(0)
    return {"estimate_ms": round(est_ms, 3),
            "flagged_channels": int(flags.sum().item()),
            "flagged_samples": int((mask == 0).sum().item()),
            "pre_step_ms": round(step_ms, 3),
            "pre_corner_turn_ms": round(ms.value / max(n.value, 1), 4)}


def forms_bench(sdd, torch, plan, xt, planes, out, ws, reps: int = 3):
    """The dedispersion stage of the step's chunk with each form of the LDS
    kernel: the matrix-core tile (the plan's default) and the vector tile,
    and whether their planes are identical."""
    import ctypes as C
    from paper_2605_03531_amd import _capi as A
    L = A.lib()
    units = plan.nchan * plan.ndm_total * plan.geometry(xt.shape[0])["n_owned"]
    keep = tuple(plan.get_tile(0))
    res, ref = {}, None
    mtile = keep if keep[0] in (5, 21) else (5, 1, 16, 1, 16, 16)
    for name, tile in (("matrix_core", mtile), ("vector", (1, 2, 8, 1, 8, 8))):
        plan.set_tile(tile)
        plan.dedisperse_search(xt, planes=planes, out=out, workspace=ws)
        torch.cuda.synchronize()
        A.check(L.sdd_profile_enable(1), "profile")
        for _ in range(reps):
            plan.dedisperse_search(xt, planes=planes, out=out, workspace=ws)
        torch.cuda.synchronize()
        ms, n = C.c_double(), C.c_int64()
        A.check(L.sdd_profile_read(A.STAGES["dedisperse"], C.byref(ms), C.byref(n)), "read")
        L.sdd_profile_enable(0)
        t = ms.value / max(n.value, 1)
        same = None
        if ref is None:
            ref = planes[0].clone()
        else:
            same = bool(torch.equal(ref, planes[0]))
        res[name] = {"tile": list(tile), "dedisperse_ms": round(t, 3),
                     "adds_per_s": round(units / t / 1e9, 2), "unit": "T adds/s",
                     "plane_equal_to_matrix_core": same}
    plan.set_tile(keep)
    del ref
    return res


def robust_bench(sdd, torch, plan, xt, planes, out, ws, reps: int = 3):
    """Search-stage time with each noise estimate, and with running-median
    de-reddening (256-sample blocks, 1280-sample window) (the step's chunk)."""
    import ctypes as C
    from paper_2605_03531_amd import _capi as A
    L = A.lib()
    res = {}
    for name, args, dered in (("moments", ("moments",), None),
                              ("clip_3sigma_3x", ("clip", 3.0, 3), None),
                              ("median_mad", ("mad",), None),
                              ("dered_256x5_moments", ("moments",), (256, 2)),
                              ("dered_256x5_median_mad", ("mad",), (256, 2))):
        plan.set_stats(*args)
        if dered is not None:
            plan.set_dereddening(*dered)
        w = ws if dered is None else None  # the de-reddening baselines need more workspace
        plan.dedisperse_search(xt, planes=planes, out=out, workspace=w)
        torch.cuda.synchronize()
        A.check(L.sdd_profile_enable(1), "profile")
        for _ in range(reps):
            plan.dedisperse_search(xt, planes=planes, out=out, workspace=w)
        torch.cuda.synchronize()
        ms, n = C.c_double(), C.c_int64()
        A.check(L.sdd_profile_read(A.STAGES["search"], C.byref(ms), C.byref(n)), "read")
        L.sdd_profile_enable(0)
        res[name] = {"search_ms": round(ms.value / max(n.value, 1), 4),
                     "candidates": int(out.ncand.cpu()[0])}
        plan.set_dereddening(0)
    plan.set_stats("moments")
    return res


def ffa_levels(m: int, p: int):
    """Depth d0 of the library's LDS sub-stacks (the shallowest whose
    sub-stacks hold <= 256 rows and <= 8192 bins): the levels above it run as
    HBM passes, two levels per pass (one single-level pass first if d0 is
    odd)."""
    fl = 0
    while (2 << fl) <= m:
        fl += 1
    d0 = 0
    while d0 < fl and (((m + (1 << d0) - 1) >> d0) * p > 8192 or ((m + (1 << d0) - 1) >> d0) > 256):
        d0 += 1
    return d0


def ffa_bench(sdd, torch, plane, n_owned: int, reps: int = 3):
    """FFA folding + boxcar search of every trial of the step's plane (2048
    series of 2^18 samples) at base periods of 1024 and 128 samples.
    Algorithmic HBM bytes per folded sample: 4 (moments) + 4 + 4 (LDS levels:
    read the rows, write the sub-stack profiles) + 20 per two-level HBM pass
    (four reads, one write) + 12 per single-level pass + 4 (boxcar read)."""
    import ctypes as C
    from paper_2605_03531_amd import _capi as A
    L = A.lib()
    series = plane[:, :n_owned]
    res = {}
    for p in (1024, 128):
        m = n_owned // p
        nb = C.c_int64()
        A.check(L.sdd_ffa_workspace_size(series.shape[0], n_owned, p, C.byref(nb)), "ws")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=plane.device)
        out = sdd.ffa_search(series, p, [1, 2, 4, 8, 16, 32, 64], 4096 * 255, workspace=ws)
        torch.cuda.synchronize()
        A.check(L.sdd_profile_enable(1), "profile")
        for _ in range(reps):
            sdd.ffa_search(series, p, [1, 2, 4, 8, 16, 32, 64], 4096 * 255, workspace=ws, out=out)
        torch.cuda.synchronize()
        ms, n = C.c_double(), C.c_int64()
        A.check(L.sdd_profile_read(A.STAGES["ffa"], C.byref(ms), C.byref(n)), "read")
        L.sdd_profile_enable(0)
        t = ms.value / max(n.value, 1)
        d0 = ffa_levels(m, p)
        nel = series.shape[0] * m * p
        by = nel * (16 + 20 * (d0 // 2) + 12 * (d0 % 2))
        best, _, _ = out.host()
        res[f"period_{p}"] = {"m": m, "hbm_levels": d0, "hbm_passes": d0 // 2 + d0 % 2,
                              "ms": round(t, 4),
                              "gsamples_per_s": round(nel / t / 1e6, 1),
                              "algorithmic_bytes": by, "gbps": round(by / t / 1e6, 1),
                              "max_snr": round(float(best["snr"].max()), 2)}
        del ws
    return res


def serve_bench(sdd, torch, nbeams: int, sat_chunks: int, rt_periods: int, max_batch: int,
                nstreams: int, per_item: bool = True, chans=(1024, 2048, 4096)):
    """Streaming server with nbeams beams (channel counts from `chans` by beam
    index), 2^16-sample chunks, 2048 DM trials 0-1000, widths 1..64.

    Saturated run: every beam submits sat_chunks chunks as fast as the rings
    allow; capacity = beams x stream seconds / wall seconds. Real-time run:
    chunks arrive at the real cadence (5.369 s per chunk) with the beams'
    phases spread over one period; latency = results on host minus the submit
    that completed the chunk's input (p50/p99 over the measured periods)."""
    import synth
    N = 1 << 16
    t_samp = 81.92e-6
    period = N * t_samp
    chans = list(chans)
    dms = np.linspace(0.0, 1000.0, 2048)
    plans = {C: sdd.Plan(np.linspace(750.0, 550.0, C), t_samp, dm_list=dms, widths=WIDTHS,
                         cand_block=1024, threshold=7.0, layout="time") for C in chans}
    pool_n = 3
    pools = {}
    for C in chans:
        x = synth.filterbank(900 + C, C, pool_n * N, 128.0, 16.0)
        pools[C] = torch.from_numpy(synth.to_time_major(x)).to("cuda:0")
    beam_c = [chans[b % len(chans)] for b in range(nbeams)]

    def run(chunks_per_beam, realtime, measure_from):
        srv = sdd.Server(hbm_budget=250 << 30, max_beams=nbeams, nstreams=nstreams,
                         max_batch=max_batch, ring_chunks=2, cap=4096, per_item=per_item)
        streams = [srv.open(plans[beam_c[b]], N, tag=b) for b in range(nbeams)]
        events = []
        for b in range(nbeams):
            phase = (b / nbeams) * period if realtime else 0.0
            for k in range(chunks_per_beam):
                events.append((phase + k * period if realtime else k, b, k))
        events.sort()
        res = []
        t0 = time.perf_counter()
        for when, b, k in events:
            if realtime:
                while True:
                    dt = t0 + when - time.perf_counter()
                    if dt <= 0:
                        break
                    res += srv.poll(256, timeout_us=int(min(dt, 0.05) * 1e6))
            C = beam_c[b]
            chunk = pools[C][(k % pool_n) * N:(k % pool_n + 1) * N]
            while streams[b].submit(chunk) != 0:
                res += srv.poll(256, timeout_us=2000)
        want = sum((chunks_per_beam * N - plans[beam_c[b]].overlap) // N for b in range(nbeams))
        while len(res) < want:
            got = srv.poll(256, timeout_us=200000)
            if not got and time.perf_counter() - t0 > 600:
                break
            res += got
        wall = time.perf_counter() - t0
        stats = srv.stats()
        srv.close()
        lat = [(r["t_done_ns"] - r["t_ready_ns"]) * 1e-9 for r in res if r["chunk"] >= measure_from]
        return res, wall, stats, lat

    log(f"serving: saturated run, {nbeams} beams x {sat_chunks} chunks")
    res, wall, stats, _ = run(sat_chunks, False, 0)
    outputs = len(res)
    stream_s = outputs * period
    capacity = stream_s / wall  # real-time beams the GPU sustains
    log(f"serving: {outputs} chunk results in {wall:.2f} s; capacity {capacity:.1f} beams; "
        f"{stats['batches']} batches")
    out = {"beams": nbeams, "chunk_samples": N, "chunk_seconds": round(period, 4),
           "channel_mix": ("/".join(map(str, chans)) + f" by beam index mod {len(chans)}"
                           if len(chans) > 1 else f"{chans[0]} on every beam"),
           "ndm": 2048, "widths": WIDTHS,
           "max_batch": max_batch, "slots": nstreams,
           "batch_launch": "one grid launch per chunk" if per_item else "persistent multi-chunk",
           "saturated": {"chunks_per_beam": sat_chunks, "results": outputs,
                         "wall_s": round(wall, 3), "real_time_beams_capacity": round(capacity, 1),
                         "rtf_per_beam": round(capacity / nbeams, 3)}}
    if rt_periods > 0:
        warm = 3  # output chunk k needs input chunks 0..k+2
        log(f"serving: real-time run, {rt_periods} periods after warm-up")
        res, wall, stats, lat = run(warm + rt_periods, True, 1)
        lat = np.array(lat)
        out["real_time"] = {"periods": warm + rt_periods, "results_measured": int(len(lat)),
                            "p50_latency_s": round(float(np.percentile(lat, 50)), 4) if len(lat) else None,
                            "p99_latency_s": round(float(np.percentile(lat, 99)), 4) if len(lat) else None,
                            "max_latency_s": round(float(lat.max()), 4) if len(lat) else None,
                            "kept_up": bool(len(lat) and float(np.percentile(lat, 99)) < period)}
        log(f"serving: p50 {out['real_time']['p50_latency_s']} s, p99 {out['real_time']['p99_latency_s']} s")
    return out


def dedisp_roofline(tile, achieved: float, ceil):
    """Roofline of the dedispersion launch for the tile shape it ran with.
    achieved: algorithmic adds per second (T adds/s, one per channel x trial
    x sample)."""
    mfma = tile[0] == 5
    peak = MFMA_PEAK_TOPS if mfma else ALU_PEAK_TOPS
    rf = {"bound": "mfma" if mfma else "alu", "kernel": "dedisperse", "tile": list(tile),
          "achieved": round(achieved, 3), "peak": round(peak, 1), "unit": "TOP/s",
          "frac": round(achieved / peak, 4), "traffic": MEASURED_TRAFFIC.get(tile)}
    if mfma:
        rf["peak_derivation"] = (f"dense int8 MFMA {MFMA_PEAK_POPS} POP/s / {MFMA_OPS_PER_ADD} "
                                 "MFMA ops per add (v_mfma_i32_16x16x64_i8: 32768 ops for "
                                 "2 channels x 256 samples)")
        rf["mfma"] = {"achieved_pops": round(achieved * MFMA_OPS_PER_ADD / 1e3, 3),
                      "peak_pops": MFMA_PEAK_POPS,
                      "frac": round(achieved * MFMA_OPS_PER_ADD / 1e3 / MFMA_PEAK_POPS, 4)}
    else:
        rf["peak_derivation"] = "256 CUs x 64 lanes x 2.4 GHz x 2 adds (v_add3_u32)"
    lds_bpa = LDS_BYTES_PER_ADD.get(tile)
    lds_peak = LDS_PEAK_TBPS
    if ceil:
        lds_peak = ceil["ds_read_b128"]["bytes_per_clk_cu"] * 256 * 2.4e9 / 1e12
    if lds_bpa:
        rf["lds"] = {"bytes_per_add": round(lds_bpa, 4),
                     "achieved": round(achieved * lds_bpa, 2), "peak": round(lds_peak, 1),
                     "unit": "TB/s", "frac": round(achieved * lds_bpa / lds_peak, 4),
                     "peak_source": ("ds_read_b128 rate measured by the ceiling probe" if ceil
                                     else "stored ds_read_b128 rate")}
    if ceil and mfma and "v_mfma_i32_16x16x64_i8" in ceil:
        # the measured matrix-instruction rate x 512 adds per instruction
        rate = ceil["v_mfma_i32_16x16x64_i8"]["wave_instr_per_clk_cu"]
        ic = rate * 512 * 256 * 2.4e9 / 1e12
        rf["issue"] = {"adds_per_mfma_instr": 512, "mfma_instr_per_clk_cu": rate,
                       "ceiling": round(ic, 2), "unit": "TOP/s", "frac": round(achieved / ic, 4)}
    elif ceil and tile in ADDS_PER_VALU:
        # adds per VALU instruction (SQ counters of this tile) x the measured
        # VOP3 issue rate
        rate = ceil["v_add3_u32"]["wave_instr_per_clk_cu"]
        ic = ADDS_PER_VALU[tile] * rate * 256 * 2.4e9 / 1e12
        rf["issue"] = {"adds_per_valu_instr": ADDS_PER_VALU[tile],
                       "valu_instr_per_clk_cu": rate, "ceiling": round(ic, 2),
                       "unit": "TOP/s", "frac": round(achieved / ic, 4)}
    return rf


def probe_ceilings():
    """VALU and LDS rates of this GPU from the ceiling probe built with the
    library (paper_2605_03531_amd/probe/ceilings.hip), or None."""
    exe = os.path.join(ROOT, "paper_2605_03531_amd", "probe", "sdd_ceilings")
    try:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        if r.returncode == 0:
            return json.loads(r.stdout.strip().splitlines()[-1])
        log(f"ceiling probe failed: {r.stderr.strip()[-300:]}")
    except (OSError, subprocess.TimeoutExpired, ValueError) as e:
        log(f"ceiling probe not run: {e}")
    return None


def normal_u8_device(torch, rows: int, cols: int, mean: float, std: float, seed: int):
    """Seeded clip(round(N(mean, std)), 0, 255) bytes made on the device in
    row blocks (the integer path's timing does not depend on the values)."""
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(seed)
    x = torch.empty((rows, cols), dtype=torch.uint8, device="cuda:0")
    for r0 in range(0, rows, 1 << 16):
        r1 = min(rows, r0 + (1 << 16))
        v = torch.randn((r1 - r0, cols), generator=gen, device="cuda:0") * std + mean
        x[r0:r1] = v.round_().clamp_(0, 255).to(torch.uint8)
        del v
    return x


def multi_range_bench(sdd, torch, steps: int, warmup: int):
    """The multi-range workload: 4096 channels 750-550 MHz, 81.92 us,
    2^19 owned samples + overlap, five DM ranges (0-100/0.1 dec 1,
    100-300/0.2 dec 2, 300-700/0.5 dec 4, 700-1500/1 dec 8, 1500-3000/2
    dec 16), boxcar widths 1..256, threshold 7; spectra input N(128, 16).
    One step = corner turn, decimation, five planes, search. Throughput in
    each range's own samples (sum_r C ndm_r N_r) and at the native rate
    (C ndm N); HBM roofline lines of the corner turn and the decimation."""
    import ctypes as C
    import synth
    from paper_2605_03531_amd import _capi as A
    L = A.lib()
    widths = [1 << k for k in range(9)]
    f = np.linspace(750.0, 550.0, 4096)
    plan = sdd.Plan(f, 81.92e-6, ranges=synth.MULTI_RANGES, widths=widths, cand_block=1024,
                    threshold=7.0, layout="time")
    T = (1 << 19) + plan.overlap
    g = plan.geometry(T)
    x = normal_u8_device(torch, T, 4096, 128.0, 16.0, 3)
    planes = plan.alloc_planes(T)
    out = plan.alloc_search_out(1 << 20)
    ws = plan.workspace(T)
    side = torch.cuda.Stream()

    def step():
        plan.dedisperse_search(x, planes=planes, out=out, workspace=ws, stream=side)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    A.check(L.sdd_profile_enable(1), "profile")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    stage = {}
    for name, sid in A.STAGES.items():
        if name in ("sift", "ffa"):
            continue
        ms, n = C.c_double(), C.c_int64()
        A.check(L.sdd_profile_read(sid, C.byref(ms), C.byref(n)), "profile_read")
        stage[name] = ms.value / steps            # per step, all launches of the stage
    L.sdd_profile_enable(0)
    ndm = plan.ndm
    own = sum(4096 * ndm[r] * g["n_owned_r"][r] for r in range(plan.nranges))
    native = 4096 * plan.ndm_total * g["n_owned"]
    decs = sorted({d for d in plan.decimation if d > 1})
    dec_bytes = 4096 * T + sum(2 * 4096 * (T // d) for d in decs)
    ct_bytes = 2 * 4096 * T
    dd_ms = stage["dedisperse"]
    res = {"workload": "multi-range: 4096 ch 750-550 MHz, 81.92 us, 2^19 owned samples, DM "
                       "0-100/0.1, 100-300/0.2 dec 2, 300-700/0.5 dec 4, 700-1500/1 dec 8, "
                       "1500-3000/2 dec 16, widths 1..256, spectra uint8 N(128,16)",
           "ndm": list(ndm), "n_owned_r": g["n_owned_r"], "nsamp_in": T,
           "tiles": [list(plan.get_tile(r)) for r in range(plan.nranges)],
           "ms_per_step": round(dt * 1e3, 3),
           "value_range_own": round(own / dt / 1e9, 2),
           "value_native_rate": round(native / dt / 1e9, 2), "unit": UNIT,
           "stage_ms": {k: round(v, 4) for k, v in stage.items()},
           "dedisperse_adds_per_s": round(own / (dd_ms / 1e3) / 1e12, 3),
           "roofline_decimate": {"bound": "hbm", "bytes": dec_bytes,
                                 "achieved_gbps": round(dec_bytes / stage["decimate"] / 1e6, 1),
                                 "peak_gbps": 8000.0,
                                 "frac": round(dec_bytes / stage["decimate"] / 1e6 / 8000.0, 4)},
           "roofline_corner_turn": {"bound": "hbm", "bytes": ct_bytes,
                                    "achieved_gbps": round(ct_bytes / stage["corner_turn"] / 1e6,
                                                           1),
                                    "peak_gbps": 8000.0,
                                    "frac": round(ct_bytes / stage["corner_turn"] / 1e6 / 8000.0,
                                                  4)},
           "candidates": int(out.ncand.cpu()[0])}
    res["uint16_forms"] = uint16_forms(torch, plan, step, planes)
    log(f"multi-range: {res}")
    del x, planes, out, ws
    return res


def uint16_forms(torch, plan, step, planes, reps: int = 2):
    """The multi-range step's dedispersion stage with the decimated (uint16)
    ranges in the four-copy vector form (their default) and in the two-copy
    vector form, and whether those ranges' planes are identical."""
    import ctypes as C
    from paper_2605_03531_amd import _capi as A
    L = A.lib()
    keep = [tuple(plan.get_tile(r)) for r in range(plan.nranges)]
    u16 = [r for r in range(plan.nranges) if plan.decimation[r] > 1]
    res, ref = {}, None
    for name, tile in (("four_copy", None), ("two_copy", (1, 2, 8, 1, 8, 4))):
        for r in u16:
            plan.set_tile(tile if tile is not None else keep[r], r)
        step()
        torch.cuda.synchronize()
        A.check(L.sdd_profile_enable(1), "profile")
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        ms, n = C.c_double(), C.c_int64()
        A.check(L.sdd_profile_read(A.STAGES["dedisperse"], C.byref(ms), C.byref(n)), "read")
        L.sdd_profile_enable(0)
        same = None
        if ref is None:
            ref = [planes[r].clone() for r in u16]
        else:
            same = all(bool(torch.equal(ref[k], planes[r])) for k, r in enumerate(u16))
        res[name] = {"tiles": [list(plan.get_tile(r)) for r in u16],
                     "dedisperse_ms": round(ms.value / reps, 3),
                     "planes_equal_to_four_copy": same}
    for r in u16:
        plan.set_tile(keep[r], r)
    res["note"] = ("dedispersion of the whole step (range 0 unchanged in both); only the "
                   "decimated ranges' tiles differ")
    del ref
    return res


def batch_bench(sdd, torch, nbeams: int):
    """nbeams beams of 4096 channels with owned lengths U[2^16, 2^18], 2048
    trials 0-1000, widths 1..64: per-beam dedisperse_search calls vs one
    batch call (persistent multi-beam launch) vs its graph replay vs the graph
    replay of per-(beam, range) grid launches. Inputs are
    uniform random bytes made on the device (the integer path's timing does
    not depend on the values)."""
    import synth
    params = synth.batched_beams(nbeams=nbeams)
    f = np.linspace(750.0, 550.0, 4096)
    plan = sdd.Plan(f, 81.92e-6, dm_list=np.linspace(0.0, 1000.0, 2048), widths=WIDTHS,
                    cand_block=1024, threshold=7.0, layout="time")
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(4)
    xs, outs = [], []
    for n, _, _ in params:
        xs.append(torch.randint(0, 256, (n + plan.overlap, 4096), dtype=torch.uint8,
                                device="cuda:0", generator=gen))
        outs.append(plan.alloc_search_out(4096))
    units = sum(4096 * 2048 * n for n, _, _ in params)
    side = torch.cuda.Stream()
    res = {"beams": nbeams, "nchan": 4096, "ndm": 2048, "owned_total": int(sum(n for n, _, _ in params))}

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    wss = [plan.workspace(x.shape[0], with_planes=True) for x in xs[:1]]
    ws_one = plan.workspace(max(x.shape[0] for x in xs), with_planes=True)

    def per_beam():
        for x, o in zip(xs, outs):
            plan.dedisperse_search(x, out=o, workspace=ws_one, stream=side)
    t = timed(per_beam)
    res["per_beam_launches"] = {"seconds": round(t, 4), "value": round(units / t / 1e9, 2)}
    del wss, ws_one
    batch = sdd.Batch([(plan, x, None, o) for x, o in zip(xs, outs)])
    ws = batch.workspace()
    t = timed(lambda: batch.run(workspace=ws, stream=side))
    res["persistent_batch"] = {"seconds": round(t, 4), "value": round(units / t / 1e9, 2)}
    t = timed(lambda: batch.run(workspace=ws, graph=True, stream=side))
    res["graph_replay"] = {"seconds": round(t, 4), "value": round(units / t / 1e9, 2)}
    # one grid launch per (beam, range), the whole batch captured and replayed as a HIP graph
    t = timed(lambda: batch.run(workspace=ws, per_item=True, graph=True, stream=side))
    res["per_item_graph_replay"] = {"seconds": round(t, 4), "value": round(units / t / 1e9, 2)}
    res["unit"] = UNIT
    log(f"batch: {res}")
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-rows", type=int, default=32,
                    help="DM trials of the oracle's bounded CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the streaming-server run")
    ap.add_argument("--serve-beams", type=int, default=160)
    ap.add_argument("--serve-chunks", type=int, default=4, help="chunks per beam, saturated run")
    ap.add_argument("--serve-periods", type=int, default=5,
                    help="measured real-time periods, mixed channel counts")
    ap.add_argument("--serve-periods-4096", type=int, default=20,
                    help="measured real-time periods, every beam at 4096 channels")
    ap.add_argument("--no-multi-range", action="store_true", help="skip the multi-range run")
    ap.add_argument("--serve-batch", type=int, default=16)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-beams run")
    ap.add_argument("--only-batch", action="store_true",
                    help="run only the batched-beams comparison (for profiling its launches); "
                         "prints its JSON object")
    ap.add_argument("--only-multi-range", action="store_true",
                    help="run only the multi-range workload (for profiling its kernels); prints "
                         "its JSON object")
    ap.add_argument("--only-step", action="store_true",
                    help="run only the full-band step (no ceiling probe, no extension rows, "
                         "no CPU baseline, serving, batch or multi-range runs: for profiling "
                         "its kernels); prints its JSON line")
    ap.add_argument("--tile", default="",
                    help="dedispersion tile of the full-band step as kind,D,WD,WT,pairs,CS "
                         "(default: the plan's choice, the first fitting menu shape)")
    ap.add_argument("--batch-beams", type=int, default=32)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy 1 GiB device-to-device three times "
                         "(a kernel of known traffic for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: beams shard across GPUs with no exchange, so "
              "whole-job throughput at N GPUs is N independent copies of this run; "
              "only the one-GPU run is measured.", file=sys.stderr)
        return 2

    if args.only_batch or args.only_multi_range:
        import torch
        import paper_2605_03531_amd as sdd
        if args.only_batch:
            print(json.dumps({"batched": batch_bench(sdd, torch, args.batch_beams)}), flush=True)
        else:
            print(json.dumps({"multi_range": multi_range_bench(sdd, torch, args.steps,
                                                               args.warmup)}), flush=True)
        return 0
    # the probe runs in its own process before this one touches the GPU
    ceil = None if args.only_step else probe_ceilings()
    log(f"ceilings: {ceil}")

    import torch
    import synth
    import paper_2605_03531_amd as sdd
    from paper_2605_03531_amd import _capi as A

    dev = torch.device("cuda:0")
    log("generating the full-band input")

    def delay_fn(f, dms, ts):
        return sdd.Plan(f, ts, dm_list=dms).delays(0)

    w = synth.full_band(delay_fn, widths=WIDTHS)
    plan = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=WIDTHS, cand_block=1024,
                    threshold=7.0, layout="time")
    if args.tile:
        plan.set_tile(tuple(int(v) for v in args.tile.split(",")))
    T = w.nsamp
    g = plan.geometry(T)
    n_owned = g["n_owned"]
    xt = torch.from_numpy(synth.to_time_major(w.x)).to(dev)
    planes = plan.alloc_planes(T)
    out = plan.alloc_search_out(1 << 20)
    ws = plan.workspace(T)
    stream = torch.cuda.Stream(device=dev)
    log(f"plan: {plan.nchan} ch, {plan.ndm_total} DMs, overlap {plan.overlap}, owned {n_owned}, "
        f"tile {plan.get_tile(0)}")

    def step():
        plan.dedisperse_search(xt, planes=planes, out=out, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warm-up done")
    L = A.lib()
    A.check(L.sdd_profile_enable(1), "profile")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    import ctypes as C
    stage = {}
    for name, sid in A.STAGES.items():
        if name == "sift":  # not part of the step; measured separately below
            continue
        ms, n = C.c_double(), C.c_int64()
        A.check(L.sdd_profile_read(sid, C.byref(ms), C.byref(n)), "profile_read")
        stage[name] = (ms.value / n.value if n.value else 0.0, n.value)
    L.sdd_profile_enable(0)
    ms_step = (t1 - t0) / args.steps * 1e3
    units = plan.nchan * plan.ndm_total * n_owned
    value = units / (ms_step / 1e3) / 1e9
    dd_ms = stage["dedisperse"][0]
    achieved = units / (dd_ms / 1e3) / 1e12 if dd_ms > 0 else 0.0
    _, _, _, ncand = out.host()
    log(f"{ms_step:.2f} ms/step; stages (avg ms): " +
        ", ".join(f"{k} {v[0]:.3f}" for k, v in stage.items()) + f"; candidates {ncand}")
    res = {
        "metric": METRIC, "value": round(value, 3), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8 in, u32 exact sums, f64 S/N", "data": "synthetic",
        "config": {"workload": "full-band beam: 4096 ch 750-550 MHz, t_samp 81.92 us, "
                               "2048 DM trials 0-1000, 2^18 owned samples + overlap, spectra "
                               "(time-major) uint8 input, boxcar widths 1..64",
                   "nchan": plan.nchan, "ndm": plan.ndm_total, "n_owned": n_owned,
                   "nsamp_in": T, "overlap": plan.overlap, "widths": WIDTHS,
                   "tile": list(plan.get_tile(0))},
        "stage_ms": {k: round(v[0], 4) for k, v in stage.items()},
        "roofline": None,
        "cpu_baseline": None,
        "ceilings": ceil,
    }
    res["roofline"] = dedisp_roofline(tuple(plan.get_tile(0)), achieved, ceil)
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(7)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)                     # runtime copy kernel
        for _ in range(3):
            torch.bitwise_not(src, out=dst)    # elementwise kernel, same traffic
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device copies and 3 x 1 GiB elementwise "
            "(1 GiB read + 1 GiB written each)")
        del src, dst
    if args.only_step:
        print(json.dumps(res), flush=True)
        return 0
    res["dedisperse_forms"] = forms_bench(sdd, torch, plan, xt, planes, out, ws)
    log(f"dedispersion forms: {res['dedisperse_forms']}")
    res["sift"] = sift_bench(sdd, torch, plan, out, float(w.dm_list[1] - w.dm_list[0]), 1 << 16)
    log(f"sift: {res['sift']}")
    res["rfi"] = rfi_bench(sdd, torch, plan, xt, planes, out, ws)
    log(f"rfi: {res['rfi']}")
    res["robust_stats"] = robust_bench(sdd, torch, plan, xt, planes, out, ws)
    log(f"robust statistics: {res['robust_stats']}")
    res["ffa"] = ffa_bench(sdd, torch, planes[0], n_owned)
    log(f"ffa: {res['ffa']}")
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(w, plan.delays(0), args.cpu_rows)
    res["serving"] = None
    res["serving_4096"] = None
    res["batched"] = None
    del xt, planes, ws, out
    torch.cuda.empty_cache()
    res["multi_range"] = None
    if not args.no_multi_range:
        res["multi_range"] = multi_range_bench(sdd, torch, 3, 1)
        torch.cuda.empty_cache()
    if not args.no_batch:
        res["batched"] = batch_bench(sdd, torch, args.batch_beams)
        torch.cuda.empty_cache()
    if not args.no_serve:
        res["serving"] = serve_bench(sdd, torch, args.serve_beams, args.serve_chunks,
                                     args.serve_periods, args.serve_batch, 2)
        torch.cuda.empty_cache()
        # the same loop with every beam at the full 4096 channels
        res["serving_4096"] = serve_bench(sdd, torch, args.serve_beams, args.serve_chunks,
                                          args.serve_periods_4096, args.serve_batch, 2,
                                          chans=(4096,))
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
