"""Python binding of libspotdd: the same calls as include/spotdd.h, with
argument marshalling only. PyTorch supplies device memory and the stream;
every step of the path runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import _capi as A

CAND_DTYPE = np.dtype([("range", "<i4"), ("dm_index", "<i4"), ("sample", "<i8"),
                       ("width", "<i4"), ("snr", "<f4")])
BEST_DTYPE = np.dtype([("snr", "<f4"), ("width", "<i4"), ("sample", "<i8")])
STATS_DTYPE = np.dtype([("n", "<i8"), ("s1", "<u8"), ("s2", "<u8"), ("mean", "<f8"),
                        ("std", "<f8")])
FFA_BEST_DTYPE = np.dtype([("snr", "<f4"), ("bin", "<i4"), ("width", "<i4"), ("pad", "<i4")])
assert CAND_DTYPE.itemsize == C.sizeof(A.Candidate)
assert BEST_DTYPE.itemsize == C.sizeof(A.DmBest)
assert STATS_DTYPE.itemsize == C.sizeof(A.DmStats)

LAYOUTS = {"chan": A.SDD_CHAN_MAJOR, "time": A.SDD_TIME_MAJOR}


def _torch():
    import torch
    return torch


def _stream_handle(stream, device: int) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _tile_tuple(t: A.Tile) -> Tuple[int, ...]:
    return (t.kind, t.dm_per_wave, t.waves_dm, t.waves_time, t.pairs_per_lane, t.chan_stage)


def tile_menu() -> List[Tuple[int, ...]]:
    n = C.c_int32()
    A.check(A.lib().sdd_tile_menu(None, 0, C.byref(n)), "sdd_tile_menu")
    arr = (A.Tile * n.value)()
    A.check(A.lib().sdd_tile_menu(arr, n.value, C.byref(n)), "sdd_tile_menu")
    return [_tile_tuple(t) for t in arr]


@dataclass
class SearchOut:
    best: "object"     # device uint8 tensor holding sdd_dm_best[ndm_total]
    stats: "object"    # device uint8 tensor holding sdd_dm_stats[ndm_total]
    cands: "object"    # device uint8 tensor holding sdd_candidate[cap]
    ncand: "object"    # device int32 tensor [1]

    def host(self):
        """(best, stats, candidates) as numpy structured arrays."""
        best = np.frombuffer(self.best.cpu().numpy().tobytes(), dtype=BEST_DTYPE)
        stats = np.frombuffer(self.stats.cpu().numpy().tobytes(), dtype=STATS_DTYPE)
        n = int(self.ncand.cpu()[0])
        cap = self.cands.numel() // CAND_DTYPE.itemsize
        raw = self.cands[: min(n, cap) * CAND_DTYPE.itemsize].cpu().numpy().tobytes()
        return best, stats, np.frombuffer(raw, dtype=CAND_DTYPE), n


class Plan:
    """sdd_plan: delay tables, overlap and tile choice for one filterbank
    format and DM grid (host only until the first compute call)."""

    def __init__(self, freqs_mhz: Sequence[float], t_samp: float, dm_list=None, ranges=None,
                 widths: Sequence[int] = (), cand_block: int = 1024, threshold: float = 7.0,
                 layout: str = "chan", device: int = 0):
        self._p = None
        f = np.ascontiguousarray(freqs_mhz, dtype=np.float64)
        d = A.PlanDesc()
        d.freqs_mhz = f.ctypes.data_as(C.POINTER(C.c_double))
        d.nchan = len(f)
        d.t_samp_s = float(t_samp)
        keep = [f]
        if dm_list is not None:
            dm = np.ascontiguousarray(dm_list, dtype=np.float64)
            keep.append(dm)
            d.dm_list = dm.ctypes.data_as(C.POINTER(C.c_double))
            d.ndm = len(dm)
        if ranges is not None:
            arr = (A.DmRange * len(ranges))()
            for k, (lo, hi, step, dec) in enumerate(ranges):
                arr[k] = A.DmRange(float(lo), float(hi), float(step), int(dec), 0)
            keep.append(arr)
            d.ranges = arr
            d.nranges = len(ranges)
        w = np.ascontiguousarray(list(widths), dtype=np.int32)
        keep.append(w)
        if len(w):
            d.widths = w.ctypes.data_as(C.POINTER(C.c_int32))
        d.nwidths = len(w)
        d.cand_block = int(cand_block)
        d.threshold = float(threshold)
        d.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
        d.device = int(device)
        ptr = C.c_void_p()
        A.check(A.lib().sdd_plan_create(C.byref(d), C.byref(ptr)), "sdd_plan_create")
        self._p = ptr
        self.device = int(device)
        self.layout = d.layout
        self.threshold = float(np.float32(threshold))
        info = A.PlanInfo()
        A.check(A.lib().sdd_plan_query(self._p, C.byref(info)), "sdd_plan_query")
        self.nchan = info.nchan
        self.nranges = info.nranges
        self.ndm_total = info.ndm_total
        self.nwidths = info.nwidths
        self.w_max = info.w_max
        self.cand_block = info.cand_block
        self.overlap = int(info.overlap)
        self.ndm = [info.ndm[r] for r in range(self.nranges)]
        self.dm_offset = [info.dm_offset[r] for r in range(self.nranges)]
        self.decimation = [info.decimation[r] for r in range(self.nranges)]
        self.max_delay = [info.max_delay[r] for r in range(self.nranges)]

    # -- host queries -------------------------------------------------
    def close(self) -> None:
        if self._p is not None:
            A.lib().sdd_plan_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._p

    def set_stats(self, mode: str = "moments", k: float = 3.0, iters: int = 3) -> None:
        """Noise estimate of the search's S/N: "moments" (default), "clip"
        (sigma-clipped, k and iters) or "mad" (median and 1.4826 * MAD)."""
        m = {"moments": A.SDD_STATS_MOMENTS, "clip": A.SDD_STATS_CLIPPED,
             "mad": A.SDD_STATS_MEDIAN_MAD}[mode]
        A.check(A.lib().sdd_plan_set_stats(self._p, m, float(k), int(iters)),
                "sdd_plan_set_stats")

    def set_dereddening(self, block: int = 0, half: int = 0) -> None:
        """Running-median de-reddening of the searched series: each block of
        `block` samples has the lower median of blocks k-half..k+half
        subtracted (re-centred at half the full scale). block=0 turns it off."""
        A.check(A.lib().sdd_plan_set_dereddening(self._p, int(block), int(half)),
                "sdd_plan_set_dereddening")

    def delays(self, r: int = 0) -> np.ndarray:
        out = np.empty((self.ndm[r], self.nchan), dtype=np.int32)
        A.check(A.lib().sdd_plan_delays(self._p, r, out.ctypes.data_as(C.POINTER(C.c_int32))),
                "sdd_plan_delays")
        return out

    def dms(self, r: int = 0) -> np.ndarray:
        out = np.empty(self.ndm[r], dtype=np.float64)
        A.check(A.lib().sdd_plan_dms(self._p, r, out.ctypes.data_as(C.POINTER(C.c_double))),
                "sdd_plan_dms")
        return out

    def geometry(self, nsamp_in: int) -> dict:
        g = A.Geometry()
        A.check(A.lib().sdd_plan_geometry(self._p, int(nsamp_in), C.byref(g)), "sdd_plan_geometry")
        R = self.nranges
        return {"nsamp_in": g.nsamp_in, "overlap": g.overlap, "n_owned": g.n_owned,
                "n_owned_r": [g.n_owned_r[r] for r in range(R)],
                "plane_cols": [g.plane_cols[r] for r in range(R)],
                "ncells": [g.ncells[r] for r in range(R)],
                "workspace_bytes": g.workspace_bytes,
                "workspace_bytes_planes": g.workspace_bytes_planes}

    def get_tile(self, r: int = 0) -> Tuple[int, ...]:
        t = A.Tile()
        A.check(A.lib().sdd_plan_get_tile(self._p, r, C.byref(t)), "sdd_plan_get_tile")
        return _tile_tuple(t)

    def set_tile(self, tile: Sequence[int], r: int = -1) -> None:
        t = A.Tile(*[int(v) for v in tile])
        A.check(A.lib().sdd_plan_set_tile(self._p, r, C.byref(t)), "sdd_plan_set_tile")

    def autotune(self, nsamp_in: int, cache_path: Optional[str] = None, stream=None) -> None:
        """Times the fitting tile shapes on the device and keeps the fastest."""
        path = cache_path.encode() if cache_path else None
        A.check(A.lib().sdd_autotune(self._p, int(nsamp_in), path,
                                     _stream_handle(stream, self.device)), "sdd_autotune")

    # -- device buffers -----------------------------------------------
    def workspace(self, nsamp_in: int, with_planes: bool = False):
        torch = _torch()
        g = self.geometry(nsamp_in)
        n = g["workspace_bytes_planes" if with_planes else "workspace_bytes"]
        return torch.empty(max(n, 1), dtype=torch.uint8, device=f"cuda:{self.device}")

    def alloc_planes(self, nsamp_in: int, pitch_align: int = 64):
        torch = _torch()
        g = self.geometry(nsamp_in)
        out = []
        for r in range(self.nranges):
            cols = g["plane_cols"][r]
            pitch = (cols + pitch_align - 1) // pitch_align * pitch_align
            out.append(torch.empty((self.ndm[r], pitch), dtype=torch.int32,
                                   device=f"cuda:{self.device}"))
        return out

    def alloc_search_out(self, cap: int = 65536) -> SearchOut:
        torch = _torch()
        dev = f"cuda:{self.device}"
        return SearchOut(
            torch.empty(self.ndm_total * BEST_DTYPE.itemsize, dtype=torch.uint8, device=dev),
            torch.empty(self.ndm_total * STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev),
            torch.empty(max(cap, 1) * CAND_DTYPE.itemsize, dtype=torch.uint8, device=dev),
            torch.zeros(1, dtype=torch.int32, device=dev))

    # -- compute ------------------------------------------------------
    def _input(self, x):
        if x.dtype.itemsize != 1 or x.dim() != 2 or x.stride(1) != 1:
            raise ValueError("input must be a 2-D uint8 tensor with unit inner stride")
        if self.layout == A.SDD_CHAN_MAJOR:
            if x.shape[0] != self.nchan:
                raise ValueError("channel-major input must be [nchan][nsamp]")
            return x.shape[1], x.stride(0)
        if x.shape[1] != self.nchan:
            raise ValueError("time-major input must be [nsamp][nchan]")
        return x.shape[0], x.stride(0)

    def _planes(self, planes):
        if len(planes) != self.nranges:
            raise ValueError("one plane per DM range")
        ptrs = (C.c_void_p * self.nranges)(*[p.data_ptr() for p in planes])
        pitch = (C.c_int64 * self.nranges)(*[p.stride(0) for p in planes])
        return ptrs, pitch

    def dedisperse(self, x, planes=None, workspace=None, stream=None):
        nsamp, pitch = self._input(x)
        if planes is None:
            planes = self.alloc_planes(nsamp)
        if workspace is None:
            workspace = self.workspace(nsamp)
        ptrs, pp = self._planes(planes)
        A.check(A.lib().sdd_dedisperse(self._p, x.data_ptr(), nsamp, pitch, ptrs, pp,
                                       workspace.data_ptr(), workspace.numel(),
                                       _stream_handle(stream, self.device)), "sdd_dedisperse")
        return planes

    def search(self, planes, nsamp_in: int, out: Optional[SearchOut] = None, cap: int = 65536,
               workspace=None, stream=None) -> SearchOut:
        if out is None:
            out = self.alloc_search_out(cap)
        if workspace is None:
            workspace = self.workspace(nsamp_in)
        ptrs, pp = self._planes(planes)
        cap = out.cands.numel() // CAND_DTYPE.itemsize
        A.check(A.lib().sdd_search_boxcar(self._p, ptrs, pp, int(nsamp_in), out.best.data_ptr(),
                                          out.stats.data_ptr(), out.cands.data_ptr(), cap,
                                          out.ncand.data_ptr(), workspace.data_ptr(),
                                          workspace.numel(),
                                          _stream_handle(stream, self.device)),
                "sdd_search_boxcar")
        return out

    def dedisperse_search(self, x, planes=None, out: Optional[SearchOut] = None,
                          cap: int = 65536, workspace=None, stream=None, lut=None,
                          time_mask=None):
        """Returns (planes or None, SearchOut). planes=None keeps the planes
        inside the workspace (not returned). lut ([nchan][256] uint8) and
        time_mask ([nsamp] uint8, 1 = keep) pre-condition the chunk first
        (sdd_dedisperse_search_pre)."""
        nsamp, pitch = self._input(x)
        pre = lut is not None or time_mask is not None
        if out is None:
            out = self.alloc_search_out(cap)
        if workspace is None:
            if pre:
                nb = C.c_int64()
                A.check(A.lib().sdd_pre_workspace_size(self._p, nsamp, 1 if planes is None else 0,
                                                       C.byref(nb)), "sdd_pre_workspace_size")
                workspace = _torch().empty(max(nb.value, 1), dtype=_torch().uint8,
                                           device=f"cuda:{self.device}")
            else:
                workspace = self.workspace(nsamp, with_planes=planes is None)
        if planes is None:
            ptrs, pp = None, None
        else:
            ptrs, pp = self._planes(planes)
        cap = out.cands.numel() // CAND_DTYPE.itemsize
        common = (out.best.data_ptr(), out.stats.data_ptr(), out.cands.data_ptr(), cap,
                  out.ncand.data_ptr(), workspace.data_ptr(), workspace.numel(),
                  _stream_handle(stream, self.device))
        if pre:
            A.check(A.lib().sdd_dedisperse_search_pre(
                self._p, x.data_ptr(), nsamp, pitch,
                None if lut is None else lut.data_ptr(),
                None if time_mask is None else time_mask.data_ptr(), ptrs, pp, *common),
                "sdd_dedisperse_search_pre")
        else:
            A.check(A.lib().sdd_dedisperse_search(self._p, x.data_ptr(), nsamp, pitch, ptrs, pp,
                                                  *common), "sdd_dedisperse_search")
        return planes, out


    def dedisperse_search_static(self, x, planes, out: SearchOut, stream=None):
        """sdd_dedisperse_search_static: the path with the library's static
        device scratch (no allocation in the call). planes may be None (kept
        in the scratch, not returned); out must be allocated beforehand."""
        nsamp, pitch = self._input(x)
        ptrs, pp = (None, None) if planes is None else self._planes(planes)
        cap = out.cands.numel() // CAND_DTYPE.itemsize
        A.check(A.lib().sdd_dedisperse_search_static(
            self._p, x.data_ptr(), nsamp, pitch, ptrs, pp, out.best.data_ptr(),
            out.stats.data_ptr(), out.cands.data_ptr(), cap, out.ncand.data_ptr(),
            _stream_handle(stream, self.device)), "sdd_dedisperse_search_static")
        return planes, out
    def rfi_estimate(self, x, median_window: int = 21, rounds: int = 2,
                     chan_sigma: float = 4.0, time_sigma: float = 3.0, stream=None):
        """Bandpass and flags of one chunk in this plan's layout
        (sdd_rfi_estimate). Returns device tensors (lut [nchan][256] uint8,
        time mask [nsamp] uint8, channel flags [nchan] int32)."""
        torch = _torch()
        nsamp, pitch = self._input(x)
        d = A.RfiDesc(int(median_window), int(rounds), float(chan_sigma), float(time_sigma))
        nb = C.c_int64()
        A.check(A.lib().sdd_rfi_workspace_size(self._p, nsamp, C.byref(nb)),
                "sdd_rfi_workspace_size")
        dev = f"cuda:{self.device}"
        ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        lut = torch.empty((self.nchan, 256), dtype=torch.uint8, device=dev)
        mask = torch.empty(nsamp, dtype=torch.uint8, device=dev)
        flags = torch.empty(self.nchan, dtype=torch.int32, device=dev)
        A.check(A.lib().sdd_rfi_estimate(self._p, x.data_ptr(), nsamp, pitch, C.byref(d),
                                         lut.data_ptr(), mask.data_ptr(), flags.data_ptr(),
                                         ws.data_ptr(), ws.numel(),
                                         _stream_handle(stream, self.device)),
                "sdd_rfi_estimate")
        return lut, mask, flags

    def sift(self, out: SearchOut, stencils=(), eps=None, min_pts: int = 0, result=None,
             workspace=None, stream=None) -> "SiftOut":
        """Candidate sifting of a search result of this plan (sdd_sift_candidates):
        stencils = [(half-size in DM, half-size in native samples), ...] applied
        in order; eps = (DM, samples) neighbourhood and min_pts the core
        threshold of the clustering (0 = no clustering)."""
        import torch
        cap = out.cands.numel() // CAND_DTYPE.itemsize
        d = A.SiftDesc()
        if len(stencils) > A.SDD_MAX_STENCILS:
            raise ValueError(f"at most {A.SDD_MAX_STENCILS} stencils")
        d.nstencils = len(stencils)
        for k, (sd, st) in enumerate(stencils):
            d.stencil_dm[k] = float(sd)
            d.stencil_t[k] = int(st)
        d.min_pts = int(min_pts)
        if eps is not None:
            d.eps_dm, d.eps_t = float(eps[0]), int(eps[1])
        dev = out.cands.device
        if result is None:
            result = SiftOut(torch.empty(cap * CAND_DTYPE.itemsize, dtype=torch.uint8, device=dev),
                             torch.zeros(1, dtype=torch.int32, device=dev),
                             torch.empty(cap, dtype=torch.int32, device=dev))
        if workspace is None:
            nb = C.c_int64()
            A.check(A.lib().sdd_sift_workspace_size(cap, C.byref(nb)), "sdd_sift_workspace_size")
            workspace = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        A.check(A.lib().sdd_sift_candidates(self._p, out.cands.data_ptr(), out.ncand.data_ptr(),
                                            cap, C.byref(d), result.cands.data_ptr(),
                                            result.n.data_ptr(), result.sizes.data_ptr(),
                                            workspace.data_ptr(), workspace.numel(),
                                            _stream_handle(stream, self.device)),
                "sdd_sift_candidates")
        return result


@dataclass
class SiftOut:
    cands: "object"    # device uint8 tensor holding sdd_candidate[cap]
    n: "object"        # device int32 tensor [1]
    sizes: "object"    # device int32 tensor [cap]

    def host(self):
        """(kept candidates as a structured array, their cluster sizes)."""
        n = int(self.n.cpu()[0])
        raw = self.cands[: n * CAND_DTYPE.itemsize].cpu().numpy().tobytes()
        return np.frombuffer(raw, dtype=CAND_DTYPE), self.sizes[:n].cpu().numpy()


@dataclass
class FfaOut:
    best: "object"      # device uint8 tensor holding sdd_ffa_best[nseries * m]
    profiles: "object"  # device int32 tensor [nseries][m][period] (uint32 bits) or None
    stats: "object"     # device uint8 tensor holding sdd_dm_stats[nseries] or None
    m: int

    def host(self):
        """(best [nseries][m] structured, profiles uint32 or None, stats or None)."""
        best = np.frombuffer(self.best.cpu().numpy().tobytes(), dtype=FFA_BEST_DTYPE)
        best = best.reshape(-1, self.m)
        prof = None if self.profiles is None else self.profiles.cpu().numpy().view(np.uint32)
        st = None if self.stats is None else np.frombuffer(self.stats.cpu().numpy().tobytes(),
                                                           dtype=STATS_DTYPE)
        return best, prof, st


def ffa_search(series, period: int, widths: Sequence[int], max_value: int, profiles: bool = False,
               stats: bool = True, workspace=None, stream=None, out: "FfaOut" = None) -> FfaOut:
    """FFA folding and boxcar search (sdd_ffa_search) of the rows of a 2-D
    device int32/uint32-bits tensor (e.g. a DM-time plane; rows may be a
    strided view with unit column stride): every row of `nsamp` columns is
    folded at the base period into m = nsamp // period profiles."""
    torch = _torch()
    if series.dim() != 2 or series.stride(1) != 1 or series.element_size() != 4:
        raise ValueError("series must be a 2-D 32-bit device tensor with unit column stride")
    ns, nsamp = series.shape
    m = nsamp // period
    dev = series.device
    w = (C.c_int32 * len(widths))(*[int(v) for v in widths])
    if out is None:
        out = FfaOut(torch.empty(ns * m * FFA_BEST_DTYPE.itemsize, dtype=torch.uint8, device=dev),
                     torch.empty((ns, m, period), dtype=torch.int32, device=dev) if profiles
                     else None,
                     torch.empty(ns * STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
                     if stats else None, m)
    if workspace is None:
        nb = C.c_int64()
        A.check(A.lib().sdd_ffa_workspace_size(ns, nsamp, int(period), C.byref(nb)),
                "sdd_ffa_workspace_size")
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    A.check(A.lib().sdd_ffa_search(dev.index or 0, series.data_ptr(), series.stride(0), ns, nsamp,
                                   int(period), int(max_value), w, len(widths),
                                   out.profiles.data_ptr() if out.profiles is not None else None,
                                   out.best.data_ptr(),
                                   out.stats.data_ptr() if out.stats is not None else None,
                                   workspace.data_ptr(), workspace.numel(),
                                   _stream_handle(stream, dev.index or 0)),
            "sdd_ffa_search")
    return out


def plane_host(plane, cols: int) -> np.ndarray:
    """Device int32 plane -> host uint32 [ndm][cols] (the defined columns)."""
    return plane[:, :cols].cpu().numpy().view(np.uint32)


class Batch:
    """A set of chunks (beams) dedispersed and searched in one call
    (sdd_batch_dedisperse_search). items: list of (plan, x, planes, out);
    planes may be None (kept in the workspace), out a SearchOut or None for
    plane-only plans."""

    def __init__(self, items):
        self._items = list(items)
        n = len(self._items)
        self._arr = (A.BatchItem * n)()
        self._keep = []
        for k, (plan, x, planes, out) in enumerate(self._items):
            nsamp, pitch = plan._input(x)
            it = self._arr[k]
            it.plan = plan.handle
            it.d_in = x.data_ptr()
            it.nsamp_in = nsamp
            it.in_pitch = pitch
            if planes is not None:
                ptrs, pp = plan._planes(planes)
                self._keep += [ptrs, pp]
                it.d_planes = C.cast(ptrs, C.POINTER(C.c_void_p))
                it.plane_pitch = C.cast(pp, C.POINTER(C.c_int64))
            if out is not None:
                it.d_best = out.best.data_ptr()
                it.d_stats = out.stats.data_ptr()
                it.d_cands = out.cands.data_ptr()
                it.cap = out.cands.numel() // CAND_DTYPE.itemsize
                it.d_ncand = out.ncand.data_ptr()
        self.device = self._items[0][0].device

    def workspace_bytes(self) -> int:
        b = C.c_int64()
        A.check(A.lib().sdd_batch_workspace_size(self._arr, len(self._items), C.byref(b)),
                "sdd_batch_workspace_size")
        return b.value

    def workspace(self):
        torch = _torch()
        return torch.empty(self.workspace_bytes(), dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    def run(self, workspace=None, per_item: bool = False, graph: bool = False, stream=None):
        if workspace is None:
            workspace = self.workspace()
        flags = (A.SDD_BATCH_PER_ITEM if per_item else 0) | (A.SDD_BATCH_GRAPH if graph else 0)
        A.check(A.lib().sdd_batch_dedisperse_search(self._arr, len(self._items), flags,
                                                    workspace.data_ptr(), workspace.numel(),
                                                    _stream_handle(stream, self.device)),
                "sdd_batch_dedisperse_search")
        return workspace


class Stream:
    """One beam of a Server (sdd_stream)."""

    def __init__(self, server, plan, chunk_nsamp: int, tag: int, snapshot: bytes = None):
        self.server, self.plan, self.n, self.tag = server, plan, int(chunk_nsamp), int(tag)
        h = C.c_void_p()
        if snapshot is None:
            A.check(A.lib().sdd_stream_open(server.handle, plan.handle, self.n, self.tag,
                                            C.byref(h)), "sdd_stream_open")
            self.seq = 0
        else:
            buf = C.create_string_buffer(bytes(snapshot), len(snapshot))
            A.check(A.lib().sdd_stream_restore(server.handle, plan.handle, buf, len(snapshot),
                                               self.tag, C.byref(h)), "sdd_stream_restore")
            # header: magic u64, version i32, nchan i32, N, O, submitted (i64 each)
            self.seq = int(np.frombuffer(bytes(snapshot)[32:40], dtype="<i8")[0])
        self._h = h

    def snapshot(self) -> bytes:
        """Checkpoint (sdd_stream_snapshot): the next sequence number, the next
        unscheduled output chunk and the spectra it and later chunks need."""
        need = C.c_int64()
        A.check(A.lib().sdd_stream_snapshot(self._h, None, 0, C.byref(need)),
                "sdd_stream_snapshot")
        buf = C.create_string_buffer(need.value)
        A.check(A.lib().sdd_stream_snapshot(self._h, buf, need.value, C.byref(need)),
                "sdd_stream_snapshot")
        return buf.raw[:need.value]

    def submit(self, chunk, seq: Optional[int] = None) -> int:
        """Copies chunk ([n][nchan] uint8 spectra: torch tensor on the device,
        or a host array) into the ring. Returns the status code: 0, or
        SDD_EAGAIN (ring full, poll and retry); raises on other errors."""
        seq = self.seq if seq is None else int(seq)
        if chunk is None:  # only meaningful for a server in fake mode
            ptr, dev = None, 0
        elif hasattr(chunk, "data_ptr"):
            ptr, dev = chunk.data_ptr(), int(chunk.is_cuda)
        else:
            arr = np.ascontiguousarray(chunk, dtype=np.uint8)
            ptr, dev = arr.ctypes.data, 0
        st = A.lib().sdd_stream_submit(self._h, ptr, self.n, seq, dev)
        if st == A.SDD_EAGAIN:
            return st
        A.check(st, "sdd_stream_submit")
        self.seq = seq + 1
        return st

    def keep_planes(self, on: bool = True) -> None:
        """Output chunks scheduled from now on also return their DM-time
        planes (sdd_stream_keep_planes); Server.poll copies them into device
        tensors under the result's "planes"."""
        A.check(A.lib().sdd_stream_keep_planes(self._h, int(bool(on))),
                "sdd_stream_keep_planes")

    def close(self) -> None:
        if self._h is not None:
            A.check(A.lib().sdd_stream_close(self._h), "sdd_stream_close")
            self._h = None


class Server:
    """sdd_server: continuous batching of many beams on one GPU."""

    def __init__(self, hbm_budget: int, device: int = 0, max_beams: int = 256,
                 nstreams: int = 2, max_batch: int = 8, ring_chunks: int = 2, cap: int = 1024,
                 per_item: bool = True, fake_exec_us: Optional[int] = None,
                 fake_fail_every: int = 0):
        d = A.ServerDesc()
        d.hbm_budget = int(hbm_budget)
        d.device = int(device)
        d.max_beams = int(max_beams)
        d.nstreams = int(nstreams)
        d.max_batch = int(max_batch)
        d.ring_chunks = int(ring_chunks)
        d.cap = int(cap)
        d.batch_flags = A.SDD_BATCH_PER_ITEM if per_item else 0
        if fake_exec_us is not None:
            d.flags = A.SDD_SERVER_FAKE
            d.fake_exec_us = int(fake_exec_us)
            d.fake_fail_every = int(fake_fail_every)
        h = C.c_void_p()
        A.check(A.lib().sdd_server_create(C.byref(d), C.byref(h)), "sdd_server_create")
        self._h = h
        self.cap = d.cap

    @property
    def handle(self):
        return self._h

    def open(self, plan, chunk_nsamp: int, tag: int = 0) -> Stream:
        return Stream(self, plan, chunk_nsamp, tag)

    def restore(self, plan, snapshot: bytes, tag: int = 0) -> Stream:
        """Opens a beam from a Stream.snapshot() checkpoint (sdd_stream_restore)."""
        n = int(np.frombuffer(bytes(snapshot)[16:24], dtype="<i8")[0])
        return Stream(self, plan, n, tag, snapshot=snapshot)

    def footprint(self, plan, chunk_nsamp: int) -> int:
        b = C.c_int64()
        A.check(A.lib().sdd_stream_footprint(self._h, plan.handle, int(chunk_nsamp),
                                             C.byref(b)), "sdd_stream_footprint")
        return b.value

    def poll(self, max_results: int = 64, timeout_us: int = 0) -> list:
        """Finished results as dicts (host copies; released at once)."""
        arr = (A.Result * max_results)()
        n = C.c_int32()
        st = A.lib().sdd_stream_poll(self._h, arr, max_results, int(timeout_us), C.byref(n))
        if st == A.SDD_ETIMEDOUT:
            return []
        A.check(st, "sdd_stream_poll")
        out = []
        for k in range(n.value):
            r = arr[k]
            nb = r.ndm
            best = np.frombuffer(C.string_at(r.best, nb * BEST_DTYPE.itemsize), dtype=BEST_DTYPE)
            nc = min(r.ncand, self.cap)
            cands = np.frombuffer(C.string_at(r.cands, nc * CAND_DTYPE.itemsize) if nc else b"",
                                  dtype=CAND_DTYPE)
            res = {"tag": r.tag, "chunk": r.chunk, "status": r.status, "ncand": r.ncand,
                   "best": best.copy(), "cands": cands.copy(), "t_ready_ns": r.t_ready_ns,
                   "t_start_ns": r.t_start_ns, "t_done_ns": r.t_done_ns}
            if r.nplanes > 0:
                res["planes"] = self._copy_planes(r)
            out.append(res)
            A.check(A.lib().sdd_result_release(self._h, C.byref(r)), "sdd_result_release")
        return out

    def _copy_planes(self, r) -> list:
        """Device copies (int32 views of the uint32 sums, [ndm_r][plane_cols])
        of a result's kept planes, made on the current stream and waited for."""
        import torch
        dst = []
        ptrs = (C.c_void_p * A.SDD_MAX_RANGES)()
        pitch = (C.c_int64 * A.SDD_MAX_RANGES)()
        for q in range(r.nplanes):
            t = torch.empty((int(r.plane_rows[q]), int(r.plane_cols[q])), dtype=torch.int32,
                            device="cuda")
            dst.append(t)
            ptrs[q] = t.data_ptr()
            pitch[q] = int(r.plane_cols[q])
        s = torch.cuda.current_stream()
        A.check(A.lib().sdd_result_copy_planes(self._h, C.byref(r), ptrs, pitch, s.cuda_stream),
                "sdd_result_copy_planes")
        s.synchronize()
        return dst

    def stats(self) -> dict:
        s = A.ServerStats()
        A.check(A.lib().sdd_server_query(self._h, C.byref(s)), "sdd_server_query")
        return {k: getattr(s, k) for k, _ in A.ServerStats._fields_}

    def close(self) -> None:
        if self._h is not None:
            A.lib().sdd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
