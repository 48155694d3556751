"""ctypes view of include/spotdd.h: struct layouts, prototypes and the loader.

Loading fails loudly when libspotdd.so is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C  # noqa: F401
import os
import re

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libspotdd.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "spotdd.h")

SDD_MAX_RANGES = 16
SDD_MAX_WIDTHS = 32
SDD_MAX_WMAX = 8192
SDD_MAX_STENCILS = 8
SDD_STATS_MOMENTS, SDD_STATS_CLIPPED, SDD_STATS_MEDIAN_MAD = 0, 1, 2
SDD_CHAN_MAJOR, SDD_TIME_MAJOR = 0, 1

STATUS = {0: "SDD_OK", -1: "SDD_EINVAL", -2: "SDD_ERANGE", -3: "SDD_ENOMEM",
          -4: "SDD_EDEVICE", -5: "SDD_EAGAIN", -6: "SDD_ESTATE", -7: "SDD_ETIMEDOUT"}
SDD_OK, SDD_EINVAL, SDD_ERANGE, SDD_ENOMEM, SDD_EDEVICE, SDD_EAGAIN, SDD_ESTATE, SDD_ETIMEDOUT = \
    0, -1, -2, -3, -4, -5, -6, -7

i32, i64, u64, f32, f64, vp = C.c_int32, C.c_int64, C.c_uint64, C.c_float, C.c_double, C.c_void_p


class DmRange(C.Structure):
    _fields_ = [("dm_lo", f64), ("dm_hi", f64), ("dm_step", f64), ("decimation", i32),
                ("reserved", i32)]


class PlanDesc(C.Structure):
    _fields_ = [("freqs_mhz", C.POINTER(f64)), ("dm_list", C.POINTER(f64)),
                ("ranges", C.POINTER(DmRange)), ("widths", C.POINTER(i32)),
                ("t_samp_s", f64), ("nchan", i32), ("ndm", i32), ("nranges", i32),
                ("nwidths", i32), ("cand_block", i32), ("threshold", f32), ("layout", i32),
                ("device", i32)]


class PlanInfo(C.Structure):
    _fields_ = [("nchan", i32), ("nranges", i32), ("ndm_total", i32), ("nwidths", i32),
                ("w_max", i32), ("cand_block", i32), ("layout", i32), ("device", i32),
                ("overlap", i64), ("ndm", i32 * SDD_MAX_RANGES),
                ("dm_offset", i32 * SDD_MAX_RANGES), ("decimation", i32 * SDD_MAX_RANGES),
                ("max_delay", i32 * SDD_MAX_RANGES)]


class Geometry(C.Structure):
    _fields_ = [("nsamp_in", i64), ("overlap", i64), ("n_owned", i64),
                ("n_owned_r", i64 * SDD_MAX_RANGES), ("plane_cols", i64 * SDD_MAX_RANGES),
                ("ncells", i64 * SDD_MAX_RANGES), ("workspace_bytes", i64),
                ("workspace_bytes_planes", i64)]


class Candidate(C.Structure):
    _fields_ = [("range", i32), ("dm_index", i32), ("sample", i64), ("width", i32), ("snr", f32)]


class DmBest(C.Structure):
    _fields_ = [("snr", f32), ("width", i32), ("sample", i64)]


class DmStats(C.Structure):
    _fields_ = [("n", i64), ("s1", u64), ("s2", u64), ("mean", f64), ("std", f64)]


class Tile(C.Structure):
    _fields_ = [("kind", i32), ("dm_per_wave", i32), ("waves_dm", i32), ("waves_time", i32),
                ("pairs_per_lane", i32), ("chan_stage", i32)]


class BatchItem(C.Structure):
    _fields_ = [("plan", vp), ("d_in", vp), ("nsamp_in", i64), ("in_pitch", i64),
                ("d_planes", C.POINTER(vp)), ("plane_pitch", C.POINTER(i64)), ("d_best", vp),
                ("d_stats", vp), ("d_cands", vp), ("cap", i32), ("reserved", i32),
                ("d_ncand", vp)]


SDD_BATCH_PER_ITEM, SDD_BATCH_GRAPH = 1, 2
SDD_SERVER_FAKE = 1


class ServerDesc(C.Structure):
    _fields_ = [("hbm_budget", i64), ("device", i32), ("max_beams", i32), ("nstreams", i32),
                ("max_batch", i32), ("ring_chunks", i32), ("cap", i32), ("batch_flags", i32),
                ("flags", i32), ("fake_exec_us", i32), ("fake_fail_every", i32)]


class Result(C.Structure):
    _fields_ = [("tag", u64), ("chunk", i64), ("status", i32), ("ncand", i32), ("ndm", i32),
                ("reserved", i32), ("best", C.POINTER(DmBest)), ("cands", C.POINTER(Candidate)),
                ("t_ready_ns", i64), ("t_start_ns", i64), ("t_done_ns", i64), ("handle", vp),
                ("nplanes", i32), ("plane_rows", i32 * SDD_MAX_RANGES),
                ("d_planes", vp * SDD_MAX_RANGES),
                ("plane_pitch", i64 * SDD_MAX_RANGES), ("plane_cols", i64 * SDD_MAX_RANGES)]


class ServerStats(C.Structure):
    _fields_ = [("open_streams", i32), ("queued_results", i32), ("hbm_used", i64),
                ("batches", i64), ("chunks", i64), ("busy_ms", f64)]

class RfiDesc(C.Structure):
    _fields_ = [("median_window", i32), ("rounds", i32), ("chan_sigma", f64),
                ("time_sigma", f64)]


class SiftDesc(C.Structure):
    _fields_ = [("nstencils", i32), ("min_pts", i32), ("stencil_dm", f64 * SDD_MAX_STENCILS),
                ("stencil_t", i64 * SDD_MAX_STENCILS), ("eps_dm", f64), ("eps_t", i64)]

PlanP = vp

_PROTOS = {
    "sdd_abi_version": (i32, []),
    "sdd_last_error": (C.c_char_p, []),
    "sdd_status_string": (C.c_char_p, [i32]),
    "sdd_plan_create": (i32, [C.POINTER(PlanDesc), C.POINTER(vp)]),
    "sdd_plan_destroy": (i32, [vp]),
    "sdd_plan_query": (i32, [vp, C.POINTER(PlanInfo)]),
    "sdd_plan_delays": (i32, [vp, i32, C.POINTER(i32)]),
    "sdd_plan_dms": (i32, [vp, i32, C.POINTER(f64)]),
    "sdd_plan_geometry": (i32, [vp, i64, C.POINTER(Geometry)]),
    "sdd_plan_get_tile": (i32, [vp, i32, C.POINTER(Tile)]),
    "sdd_plan_set_tile": (i32, [vp, i32, C.POINTER(Tile)]),
    "sdd_tile_menu": (i32, [C.POINTER(Tile), i32, C.POINTER(i32)]),
    "sdd_plan_set_stats": (i32, [vp, i32, f64, i32]),
    "sdd_plan_set_dereddening": (i32, [vp, i32, i32]),
    "sdd_autotune": (i32, [vp, i64, C.c_char_p, vp]),
    "sdd_dedisperse": (i32, [vp, vp, i64, i64, C.POINTER(vp), C.POINTER(i64), vp, i64, vp]),
    "sdd_search_boxcar": (i32, [vp, C.POINTER(vp), C.POINTER(i64), i64, vp, vp, vp, i32, vp,
                                vp, i64, vp]),
    "sdd_dedisperse_search": (i32, [vp, vp, i64, i64, C.POINTER(vp), C.POINTER(i64), vp, vp,
                                    vp, i32, vp, vp, i64, vp]),
    "sdd_dedisperse_search_static": (i32, [vp, vp, i64, i64, C.POINTER(vp), C.POINTER(i64),
                                           vp, vp, vp, i32, vp, vp]),
    "sdd_batch_workspace_size": (i32, [C.POINTER(BatchItem), i32, C.POINTER(i64)]),
    "sdd_batch_dedisperse_search": (i32, [C.POINTER(BatchItem), i32, i32, vp, i64, vp]),
    "sdd_batch_graph_clear": (i32, []),
    "sdd_server_create": (i32, [C.POINTER(ServerDesc), C.POINTER(vp)]),
    "sdd_server_destroy": (i32, [vp]),
    "sdd_stream_footprint": (i32, [vp, vp, i64, C.POINTER(i64)]),
    "sdd_stream_open": (i32, [vp, vp, i64, u64, C.POINTER(vp)]),
    "sdd_stream_submit": (i32, [vp, vp, i64, u64, i32]),
    "sdd_stream_snapshot": (i32, [vp, vp, i64, C.POINTER(i64)]),
    "sdd_stream_restore": (i32, [vp, vp, vp, i64, u64, C.POINTER(vp)]),
    "sdd_stream_close": (i32, [vp]),
    "sdd_stream_poll": (i32, [vp, C.POINTER(Result), i32, i32, C.POINTER(i32)]),
    "sdd_result_release": (i32, [vp, C.POINTER(Result)]),
    "sdd_stream_keep_planes": (i32, [vp, i32]),
    "sdd_result_copy_planes": (i32, [vp, C.POINTER(Result), C.POINTER(vp), C.POINTER(i64),
                                     vp]),
    "sdd_server_query": (i32, [vp, C.POINTER(ServerStats)]),
    "sdd_rfi_workspace_size": (i32, [vp, i64, C.POINTER(i64)]),
    "sdd_rfi_estimate": (i32, [vp, vp, i64, i64, C.POINTER(RfiDesc), vp, vp, vp, vp, i64, vp]),
    "sdd_pre_workspace_size": (i32, [vp, i64, i32, C.POINTER(i64)]),
    "sdd_dedisperse_search_pre": (i32, [vp, vp, i64, i64, vp, vp, C.POINTER(vp), C.POINTER(i64),
                                        vp, vp, vp, i32, vp, vp, i64, vp]),
    "sdd_sift_workspace_size": (i32, [i32, C.POINTER(i64)]),
    "sdd_sift_candidates": (i32, [vp, vp, vp, i32, C.POINTER(SiftDesc), vp, vp, vp, vp, i64,
                                  vp]),
    "sdd_ffa_workspace_size": (i32, [i32, i64, i32, C.POINTER(i64)]),
    "sdd_ffa_search": (i32, [i32, vp, i64, i32, i64, i32, C.c_uint32, C.POINTER(i32), i32, vp, vp,
                             vp, vp, i64, vp]),
    "sdd_profile_enable": (i32, [i32]),
    "sdd_profile_read": (i32, [i32, C.POINTER(f64), C.POINTER(i64)]),
}
STAGES = {"corner_turn": 0, "decimate": 1, "dedisperse": 2, "search": 3, "sift": 4, "ffa": 5}

_lib = None


def header_functions() -> list:
    """Names of every function include/spotdd.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sdd_[a-z0-9_]+)\s*\(", txt)))


def lib() -> C.CDLL:
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2605_03531_amd.build` "
                "(there is no fallback implementation)")
        # torch's HIP build ships its own libamdhip64 (SONAME libamdhip64.so.7)
        # and loads it by another file name. Importing torch first maps that
        # copy, so this library's libamdhip64.so.7 dependency resolves to it
        # and the process holds a single HIP runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SddError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().sdd_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != SDD_OK:
        raise SddError(status, where)
