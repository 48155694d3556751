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
                          cap: int = 65536, workspace=None, stream=None):
        """Returns (planes or None, SearchOut). planes=None keeps the planes
        inside the workspace (not returned)."""
        nsamp, pitch = self._input(x)
        if out is None:
            out = self.alloc_search_out(cap)
        if workspace is None:
            workspace = self.workspace(nsamp, with_planes=planes is None)
        if planes is None:
            ptrs, pp = None, None
        else:
            ptrs, pp = self._planes(planes)
        cap = out.cands.numel() // CAND_DTYPE.itemsize
        A.check(A.lib().sdd_dedisperse_search(self._p, x.data_ptr(), nsamp, pitch, ptrs, pp,
                                              out.best.data_ptr(), out.stats.data_ptr(),
                                              out.cands.data_ptr(), cap, out.ncand.data_ptr(),
                                              workspace.data_ptr(), workspace.numel(),
                                              _stream_handle(stream, self.device)),
                "sdd_dedisperse_search")
        return planes, out


def plane_host(plane, cols: int) -> np.ndarray:
    """Device int32 plane -> host uint32 [ndm][cols] (the defined columns)."""
    return plane[:, :cols].cpu().numpy().view(np.uint32)
