// extern "C" compute entry points of libspotdd: argument checks, workspace
// carving and the launch sequence of one chunk (corner turn -> decimation ->
// dedispersion per range -> boxcar search).
#include <algorithm>
#include <cstring>
#include <mutex>

#include "sdd_internal.h"

namespace sdd {
const char* last_error();

sdd_status check_planes(const sdd_plan* p, const CallGeom& cg, const void* const* planes,
                        const int64_t* pitch) {
  if (!planes || !pitch) SDD_FAIL(SDD_EINVAL, "null plane array or pitch array");
  for (size_t r = 0; r < p->ranges.size(); ++r) {
    if (!planes[r]) SDD_FAIL(SDD_EINVAL, "null plane for range %zu", r);
    if (pitch[r] < cg.g.plane_cols[r])
      SDD_FAIL(SDD_EINVAL, "range %zu: plane pitch %lld < %lld columns", r, (long long)pitch[r],
               (long long)cg.g.plane_cols[r]);
  }
  return SDD_OK;
}

sdd_status check_input(const sdd_plan* p, const uint8_t* d_in, int64_t nsamp_in,
                       int64_t in_pitch) {
  if (!d_in) SDD_FAIL(SDD_EINVAL, "null input");
  if (p->layout == SDD_TIME_MAJOR && in_pitch < p->nchan)
    SDD_FAIL(SDD_EINVAL, "time-major pitch %lld < nchan %d", (long long)in_pitch, p->nchan);
  if (p->layout == SDD_CHAN_MAJOR && in_pitch < nsamp_in)
    SDD_FAIL(SDD_EINVAL, "channel-major pitch %lld < nsamp_in %lld", (long long)in_pitch,
             (long long)nsamp_in);
  return SDD_OK;
}

sdd_status prep_item(const sdd_plan* p, const CallGeom& cg, const uint8_t* d_in, int64_t nsamp_in,
                     int64_t in_pitch, uint32_t* const* planes, const int64_t* pitch, uint8_t* ws,
                     hipStream_t s, std::vector<DedispArgs>* jobs, int64_t ring_rows,
                     int64_t ring_start, const Precond* pre) {
  const WsLayout& L = cg.ws;
  const uint8_t* src = d_in;
  int64_t src_pitch = in_pitch;
  if (p->layout == SDD_TIME_MAJOR) {
    uint8_t* ct = ws + L.ct_off;
    StageTimer tm(SDD_STAGE_CORNER_TURN, s);
    SDD_HIP_TRY(launch_corner_turn(d_in, nsamp_in, in_pitch, p->nchan, ct, L.ct_pitch, s,
                                   ring_rows, ring_start, pre ? pre->lut : nullptr,
                                   pre ? pre->tmask : nullptr));
    src = ct;
    src_pitch = L.ct_pitch;
  } else if (pre && (pre->lut || pre->tmask)) {
    StageTimer tm(SDD_STAGE_CORNER_TURN, s);
    SDD_HIP_TRY(launch_precond_rows(d_in, in_pitch, nsamp_in, p->nchan, pre->lut, pre->tmask,
                                    pre->rows, pre->rows_pitch, s));
    src = pre->rows;
    src_pitch = pre->rows_pitch;
  }
  std::vector<uint16_t*> dbuf(L.decs.size());
  for (size_t k = 0; k < L.decs.size(); ++k)
    dbuf[k] = reinterpret_cast<uint16_t*>(ws + L.dec_off[k]);
  // decimations 2, 4, 8, 16 only: one pass over the uint8 rows
  bool pow2 = !L.decs.empty();
  for (int32_t d : L.decs) pow2 = pow2 && (d == 2 || d == 4 || d == 8 || d == 16);
  if (pow2) {
    DecLevels lv;
    for (size_t k = 0; k < L.decs.size(); ++k) {
      const int l = L.decs[k] == 2 ? 0 : L.decs[k] == 4 ? 1 : L.decs[k] == 8 ? 2 : 3;
      lv.out[l] = dbuf[k];
      lv.pitch[l] = L.dec_pitch[k];
      lv.len[l] = L.dec_len[k];
    }
    StageTimer tm(SDD_STAGE_DECIMATE, s);
    SDD_HIP_TRY(launch_decimate_pow2(src, src_pitch, nsamp_in, p->nchan, lv, s));
  }
  // otherwise each decimation is built from the largest smaller one that divides it
  for (size_t k = 0; k < L.decs.size() && !pow2; ++k) {
    int32_t d = L.decs[k];
    int from = -1;
    for (int j = (int)k - 1; j >= 0; --j)
      if (d % L.decs[j] == 0) {
        from = j;
        break;
      }
    StageTimer tm(SDD_STAGE_DECIMATE, s);
    if (from < 0) {
      SDD_HIP_TRY(launch_decimate(src, 1, src_pitch, p->nchan, d, dbuf[k], L.dec_pitch[k],
                                  L.dec_len[k], s));
    } else {
      SDD_HIP_TRY(launch_decimate(dbuf[from], 2, L.dec_pitch[from], p->nchan,
                                  d / L.decs[from], dbuf[k], L.dec_pitch[k], L.dec_len[k], s));
    }
  }
  for (size_t r = 0; r < p->ranges.size(); ++r) {
    const Range& R = p->ranges[r];
    DedispArgs a{};
    if (R.dec == 1) {
      a.x = src;
      a.elem_bytes = 1;
      a.x_pitch = src_pitch;
      a.x_len = nsamp_in;
    } else {
      size_t k = std::find(L.decs.begin(), L.decs.end(), R.dec) - L.decs.begin();
      a.x = dbuf[k];
      a.elem_bytes = 2;
      a.x_pitch = L.dec_pitch[k];
      a.x_len = L.dec_len[k];
    }
    a.nchan = p->nchan;
    a.delays = p->d_delays[r];
    a.ndm = R.ndm();
    a.plane = planes[r];
    a.plane_pitch = pitch[r];
    a.cols = cg.g.plane_cols[r];
    a.max_val = 255 * R.dec;
    a.tile = R.tile;
    a.span = R.tile_span;
    a.max_delay = R.max_delay;
    if (a.cols + R.max_delay > a.x_len)
      SDD_FAIL(SDD_EINVAL, "internal: range %zu input too short", r);
    jobs->push_back(a);
  }
  return SDD_OK;
}

sdd_status run_dedisperse(const sdd_plan* p, const CallGeom& cg, const uint8_t* d_in,
                          int64_t nsamp_in, int64_t in_pitch, uint32_t* const* planes,
                          const int64_t* pitch, uint8_t* ws, hipStream_t s, const Precond* pre) {
  std::vector<DedispArgs> jobs;
  sdd_status st = prep_item(p, cg, d_in, nsamp_in, in_pitch, planes, pitch, ws, s, &jobs, 0, 0,
                            pre);
  if (st != SDD_OK) return st;
  for (const auto& a : jobs) {
    StageTimer tm(SDD_STAGE_DEDISPERSE, s);
    SDD_HIP_TRY(launch_dedisperse(a, s));
  }
  return SDD_OK;
}

sdd_status run_search(const sdd_plan* p, const CallGeom& cg, const uint32_t* const* planes,
                      const int64_t* pitch, sdd_dm_best* best, sdd_dm_stats* stats,
                      sdd_candidate* cands, int32_t cap, int32_t* ncand, uint8_t* ws,
                      hipStream_t s) {
  SearchArgs a{};
  a.nranges = (int32_t)p->ranges.size();
  a.ndm_total = p->ndm_total;
  a.nwidths = (int32_t)p->widths.size();
  a.w_max = p->w_max;
  for (int32_t k = 0; k < a.nwidths; ++k) a.widths[k] = p->widths[k];
  a.cand_block = p->cand_block;
  a.threshold = p->threshold;
  a.cap = cap;
  a.max_boxcar = (int64_t)p->nchan * 255 * p->dec_max * p->w_max;
  a.max_sample = (int64_t)p->nchan * 255 * p->dec_max;
  a.stats_mode = p->stats_mode;
  a.clip_k = p->clip_k;
  a.clip_iters = p->clip_iters;
  a.robust_off = cg.ws.robust_off;
  a.dered_shift = 0;
  if (p->dered_block > 0) {
    while ((1 << a.dered_shift) < p->dered_block) ++a.dered_shift;
    a.dered_half = p->dered_half;
    a.dered_elems = (int32_t)(((int64_t)(2 * p->dered_half + 1) * p->dered_block + 63) / 64);
    a.dered_nb = (int32_t)cg.ws.dered_nb;
    a.dered_off = cg.ws.dered_off;
  }
  a.max_cells = 0;
  for (int32_t r = 0; r < a.nranges; ++r) {
    const Range& R = p->ranges[r];
    a.r[r].plane = planes[r];
    a.r[r].pitch = pitch[r];
    a.r[r].n_owned = cg.g.n_owned_r[r];
    a.r[r].ndm = R.ndm();
    a.r[r].dm_offset = R.dm_offset;
    a.r[r].ncells = (int32_t)cg.g.ncells[r];
    a.r[r].full_scale = (int32_t)std::min<int64_t>((int64_t)p->nchan * 255 * R.dec, INT32_MAX);
    a.r[r].cell_base = cg.cell_base[r];
    a.max_cells = std::max(a.max_cells, a.r[r].ncells);
  }
  a.ws = ws;
  a.cellres_off = cg.ws.cellres_off;
  a.moments_off = cg.ws.moments_off;
  a.cellbest_off = cg.ws.cellbest_off;
  a.rowcnt_off = cg.ws.rowcnt_off;
  a.rowoff_off = cg.ws.rowoff_off;
  a.best = best;
  a.stats = stats;
  a.cands = cands;
  a.ncand = ncand;
  StageTimer tm(SDD_STAGE_SEARCH, s);
  SDD_HIP_TRY(launch_search(a, s));
  return SDD_OK;
}

}  // namespace sdd

using namespace sdd;

extern "C" int32_t sdd_abi_version(void) { return SDD_ABI_VERSION; }
extern "C" const char* sdd_last_error(void) { return sdd::last_error(); }
extern "C" const char* sdd_status_string(int32_t s) {
  switch (s) {
    case SDD_OK: return "SDD_OK";
    case SDD_EINVAL: return "SDD_EINVAL";
    case SDD_ERANGE: return "SDD_ERANGE";
    case SDD_ENOMEM: return "SDD_ENOMEM";
    case SDD_EDEVICE: return "SDD_EDEVICE";
    case SDD_EAGAIN: return "SDD_EAGAIN";
    case SDD_ESTATE: return "SDD_ESTATE";
    case SDD_ETIMEDOUT: return "SDD_ETIMEDOUT";
    default: return "unknown status";
  }
}

extern "C" sdd_status sdd_dedisperse(const sdd_plan* p, const uint8_t* d_in, int64_t nsamp_in,
                                     int64_t in_pitch, uint32_t* const* d_planes,
                                     const int64_t* plane_pitch, void* d_ws, int64_t ws_bytes,
                                     void* stream) {
  clear_error();
  if (!p) SDD_FAIL(SDD_EINVAL, "null plan");
  CallGeom cg;
  sdd_status st = plan_geometry(p, nsamp_in, &cg);
  if (st != SDD_OK) return st;
  if ((st = check_input(p, d_in, nsamp_in, in_pitch)) != SDD_OK) return st;
  if ((st = check_planes(p, cg, (const void* const*)d_planes, plane_pitch)) != SDD_OK) return st;
  if (ws_bytes < cg.ws.total || (cg.ws.total > 0 && !d_ws))
    SDD_FAIL(SDD_ENOMEM, "workspace %lld bytes < %lld needed", (long long)ws_bytes,
             (long long)cg.ws.total);
  SDD_CHECK_WS_ALIGN(d_ws);
  DeviceGuard dg(p->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", p->device);
  if ((st = plan_upload(p)) != SDD_OK) return st;
  return run_dedisperse(p, cg, d_in, nsamp_in, in_pitch, d_planes, plane_pitch, (uint8_t*)d_ws,
                        (hipStream_t)stream);
}

extern "C" sdd_status sdd_search_boxcar(const sdd_plan* p, const uint32_t* const* d_planes,
                                        const int64_t* plane_pitch, int64_t nsamp_in,
                                        sdd_dm_best* d_best, sdd_dm_stats* d_stats,
                                        sdd_candidate* d_cands, int32_t cap, int32_t* d_ncand,
                                        void* d_ws, int64_t ws_bytes, void* stream) {
  clear_error();
  if (!p) SDD_FAIL(SDD_EINVAL, "null plan");
  if (p->widths.empty()) SDD_FAIL(SDD_EINVAL, "plan has no boxcar widths");
  if (!d_best || !d_ncand || cap < 0 || (cap > 0 && !d_cands))
    SDD_FAIL(SDD_EINVAL, "null best/ncand, or null candidates with cap > 0");
  CallGeom cg;
  sdd_status st = plan_geometry(p, nsamp_in, &cg);
  if (st != SDD_OK) return st;
  if ((st = check_planes(p, cg, (const void* const*)d_planes, plane_pitch)) != SDD_OK) return st;
  if (ws_bytes < cg.ws.total || !d_ws)
    SDD_FAIL(SDD_ENOMEM, "workspace %lld bytes < %lld needed", (long long)ws_bytes,
             (long long)cg.ws.total);
  SDD_CHECK_WS_ALIGN(d_ws);
  DeviceGuard dg(p->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", p->device);
  if ((st = plan_upload(p)) != SDD_OK) return st;
  return run_search(p, cg, d_planes, plane_pitch, d_best, d_stats, d_cands, cap, d_ncand,
                    (uint8_t*)d_ws, (hipStream_t)stream);
}

extern "C" sdd_status sdd_dedisperse_search(const sdd_plan* p, const uint8_t* d_in,
                                            int64_t nsamp_in, int64_t in_pitch,
                                            uint32_t* const* d_planes,
                                            const int64_t* plane_pitch, sdd_dm_best* d_best,
                                            sdd_dm_stats* d_stats, sdd_candidate* d_cands,
                                            int32_t cap, int32_t* d_ncand, void* d_ws,
                                            int64_t ws_bytes, void* stream) {
  clear_error();
  if (!p) SDD_FAIL(SDD_EINVAL, "null plan");
  if (p->widths.empty()) SDD_FAIL(SDD_EINVAL, "plan has no boxcar widths");
  if (!d_best || !d_ncand || cap < 0 || (cap > 0 && !d_cands))
    SDD_FAIL(SDD_EINVAL, "null best/ncand, or null candidates with cap > 0");
  CallGeom cg;
  sdd_status st = plan_geometry(p, nsamp_in, &cg);
  if (st != SDD_OK) return st;
  if ((st = check_input(p, d_in, nsamp_in, in_pitch)) != SDD_OK) return st;
  uint32_t* own[SDD_MAX_RANGES];
  int64_t own_pitch[SDD_MAX_RANGES];
  const bool lib_planes = (d_planes == nullptr);
  const int64_t need = lib_planes ? cg.ws.total_planes : cg.ws.total;
  if (ws_bytes < need || !d_ws)
    SDD_FAIL(SDD_ENOMEM, "workspace %lld bytes < %lld needed", (long long)ws_bytes,
             (long long)need);
  SDD_CHECK_WS_ALIGN(d_ws);
  if (lib_planes) {
    for (size_t r = 0; r < p->ranges.size(); ++r) {
      own[r] = reinterpret_cast<uint32_t*>((uint8_t*)d_ws + cg.ws.plane_off[r]);
      own_pitch[r] = cg.ws.plane_pitch[r];
    }
    d_planes = own;
    plane_pitch = own_pitch;
  } else if ((st = check_planes(p, cg, (const void* const*)d_planes, plane_pitch)) != SDD_OK) {
    return st;
  }
  DeviceGuard dg(p->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", p->device);
  if ((st = plan_upload(p)) != SDD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = run_dedisperse(p, cg, d_in, nsamp_in, in_pitch, d_planes, plane_pitch, (uint8_t*)d_ws, s);
  if (st != SDD_OK) return st;
  return run_search(p, cg, (const uint32_t* const*)d_planes, plane_pitch, d_best, d_stats,
                    d_cands, cap, d_ncand, (uint8_t*)d_ws, s);
}

// ---- allocation-free variant ------------------------------------------------
//
// The scratch of sdd_dedisperse_search_static: a device array in this module,
// one copy on each device the library runs on, held until the process ends.
// Host code never passes `scratch` itself (its host-side name is not a device
// address); it passes the address hipGetSymbolAddress returns for the device,
// looked up once per device on the entry point's first call there.

namespace {

constexpr int64_t kStaticScratchBytes = (int64_t)256 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {nullptr};

// Device address of this device's copy of `scratch` (caller has the device
// current).
sdd_status static_scratch(int device, uint8_t** out) {
  if (device < 0 || device >= kMaxDevices) SDD_FAIL(SDD_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      SDD_FAIL(SDD_EDEVICE, "static scratch address on device %d: %s", device,
               hipGetErrorString(e));
    g_scratch[device] = static_cast<uint8_t*>(ptr);
  }
  *out = g_scratch[device];
  return SDD_OK;
}

}  // namespace

extern "C" sdd_status sdd_dedisperse_search_static(const sdd_plan* p, const uint8_t* d_in,
                                                   int64_t nsamp_in, int64_t in_pitch,
                                                   uint32_t* const* d_planes,
                                                   const int64_t* plane_pitch,
                                                   sdd_dm_best* d_best, sdd_dm_stats* d_stats,
                                                   sdd_candidate* d_cands, int32_t cap,
                                                   int32_t* d_ncand, void* stream) {
  clear_error();
  if (!p) SDD_FAIL(SDD_EINVAL, "null plan");
  if (p->widths.empty()) SDD_FAIL(SDD_EINVAL, "plan has no boxcar widths");
  if (!d_best || !d_ncand || cap < 0 || (cap > 0 && !d_cands))
    SDD_FAIL(SDD_EINVAL, "null best/ncand, or null candidates with cap > 0");
  CallGeom cg;
  sdd_status st = plan_geometry(p, nsamp_in, &cg);
  if (st != SDD_OK) return st;
  if ((st = check_input(p, d_in, nsamp_in, in_pitch)) != SDD_OK) return st;
  const bool lib_planes = (d_planes == nullptr);
  const int64_t need = lib_planes ? cg.ws.total_planes : cg.ws.total;
  if (need > kStaticScratchBytes)
    SDD_FAIL(SDD_ENOMEM, "this chunk needs %lld bytes of scratch; the static scratch holds %lld",
             (long long)need, (long long)kStaticScratchBytes);
  if (!lib_planes &&
      (st = check_planes(p, cg, (const void* const*)d_planes, plane_pitch)) != SDD_OK)
    return st;
  {
    // the plan's device tables are allocated by the first regular compute
    // call; this entry point allocates nothing, so it needs them in place
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->uploaded_device != p->device)
      SDD_FAIL(SDD_ESTATE, "the plan's device tables do not exist yet: run any other compute "
                           "call with this plan first");
  }
  DeviceGuard dg(p->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", p->device);
  uint8_t* ws = nullptr;
  if ((st = static_scratch(p->device, &ws)) != SDD_OK) return st;
  uint32_t* own[SDD_MAX_RANGES];
  int64_t own_pitch[SDD_MAX_RANGES];
  if (lib_planes) {
    for (size_t r = 0; r < p->ranges.size(); ++r) {
      own[r] = reinterpret_cast<uint32_t*>(ws + cg.ws.plane_off[r]);
      own_pitch[r] = cg.ws.plane_pitch[r];
    }
    d_planes = own;
    plane_pitch = own_pitch;
  }
  hipStream_t s = (hipStream_t)stream;
  st = run_dedisperse(p, cg, d_in, nsamp_in, in_pitch, d_planes, plane_pitch, ws, s);
  if (st != SDD_OK) return st;
  return run_search(p, cg, (const uint32_t* const*)d_planes, plane_pitch, d_best, d_stats,
                    d_cands, cap, d_ncand, ws, s);
}
