// Host side of the plan: descriptor validation, the FP64 delay tables
// (Chapter 1, Eq. (1)), the exactness guards, per-call geometry and the
// workspace layout. Nothing here launches a kernel; only plan_upload touches
// the GPU (on first use by a compute call).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "k_dedisp_lds.h"
#include "sdd_internal.h"

namespace sdd {

namespace {
thread_local char g_err[1024] = {0};

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Delay of every channel at one trial DM, in samples of dec * t_samp, rounded
// half up. Written as ((K * DM) * diff) / den so it rounds exactly as the
// documented left-to-right FP64 evaluation; this file is compiled without
// floating-point contraction.
sdd_status build_delays(const std::vector<double>& freqs, double t_samp, Range& r) {
  const double ftop = *std::max_element(freqs.begin(), freqs.end());
  const double inv_top = 1.0 / (ftop * ftop);
  std::vector<double> diff(freqs.size());
  for (size_t c = 0; c < freqs.size(); ++c) diff[c] = 1.0 / (freqs[c] * freqs[c]) - inv_top;
  const double den = (double)r.dec * t_samp;
  const size_t nchan = freqs.size();
  r.delays.assign(r.dms.size() * nchan, 0);
  r.max_delay = 0;
  for (size_t i = 0; i < r.dms.size(); ++i) {
    for (size_t c = 0; c < nchan; ++c) {
      double v = kDispersionConstant * r.dms[i] * diff[c] / den;
      double d = std::floor(v + 0.5);
      if (!(d >= 0.0) || d > 1.0e9)
        SDD_FAIL(SDD_ERANGE, "delay %g samples at DM %g channel %zu is out of range", d,
                 r.dms[i], c);
      int32_t di = (int32_t)d;
      r.delays[i * nchan + c] = di;
      r.max_delay = std::max(r.max_delay, di);
    }
  }
  return SDD_OK;
}
}  // namespace

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = 0; }
const char* last_error() { return g_err; }

const std::vector<sdd_tile>& tile_menu() {
  static const std::vector<sdd_tile> menu = [] {
    std::vector<sdd_tile> m;
    for (int k = 0; k < kNumLdsShapes; ++k) {
      const LdsShape& sh = kLdsShapes[k];
      m.push_back({1 + sh.f, sh.d, sh.wd, sh.wt, 4 * sh.m, sh.cs});
    }
    m.push_back({0, 0, 0, 0, 0, 0});
    return m;
  }();
  return menu;
}

// Index of t in the LDS shape table, or -1.
int lds_shape_index(const sdd_tile& t) {
  if (t.kind < 1) return -1;
  for (int k = 0; k < kNumLdsShapes; ++k) {
    const LdsShape& sh = kLdsShapes[k];
    if (t.kind == 1 + sh.f && t.dm_per_wave == sh.d && t.waves_dm == sh.wd && t.waves_time == sh.wt &&
        t.pairs_per_lane == 4 * sh.m && t.chan_stage == sh.cs)
      return k;
  }
  return -1;
}

bool tile_in_menu(const sdd_tile& t) {
  for (const auto& m : tile_menu())
    if (std::memcmp(&m, &t, sizeof(sdd_tile)) == 0) return true;
  return false;
}

int32_t range_span(const sdd_plan* p, int32_t r, int32_t dm_tile) {
  const Range& R = p->ranges[r];
  const int32_t ndm = R.ndm(), C = p->nchan;
  int32_t span = 0;
  for (int32_t i0 = 0; i0 < ndm; i0 += dm_tile) {
    int32_t i1 = std::min(ndm, i0 + dm_tile) - 1;
    for (int32_t c = 0; c < C; ++c)
      span = std::max(span, R.delays[(size_t)i1 * C + c] - R.delays[(size_t)i0 * C + c]);
  }
  return span;
}

sdd_status check_tile_fits(const sdd_plan* p, int32_t r, const sdd_tile& t, int32_t* span_out) {
  if (!tile_in_menu(t)) SDD_FAIL(SDD_EINVAL, "tile shape not in the built menu");
  if (span_out) *span_out = 0;
  if (t.kind == 0) return SDD_OK;
  if (lds_shape_index(t) < 0) SDD_FAIL(SDD_EINVAL, "tile shape not in the built menu");
  const Range& R = p->ranges[r];
  const int es = R.dec == 1 ? 1 : 2;
  const LdsShape& sh = kLdsShapes[lds_shape_index(t)];
  if (lds_flush_period(sh, 255 * R.dec) < sh.cs)
    SDD_FAIL(SDD_EINVAL, "range %d: decimation %d is too large for 16-bit accumulation", r,
             R.dec);
  // the kernel takes a tile's first trial as its smallest delay
  for (size_t i = 1; i < R.dms.size(); ++i)
    if (R.dms[i] < R.dms[i - 1])
      SDD_FAIL(SDD_EINVAL, "range %d: the LDS kernel needs ascending trial DMs", r);
  if ((sh.f & 4) != 0 && es != 1)
    SDD_FAIL(SDD_EINVAL, "range %d: the matrix-core tile takes uint8 rows (decimation 1) only", r);
  if ((sh.f & 8) != 0 && es != 2)
    SDD_FAIL(SDD_EINVAL, "range %d: the four-copy tile takes uint16 rows (decimation > 1) only", r);
  const int32_t dt = sh.d * sh.wd, tt = lds_tile_samples(sh, es), nt = 64 * sh.wd * sh.wt;
  const int32_t span = range_span(p, r, dt);
  const int64_t win = lds_window_bytes(tt, span, es);
  const int64_t lds = lds_tile_bytes(sh, win);
  if (lds > 160 * 1024)
    SDD_FAIL(SDD_EINVAL, "range %d: delay span %d needs %lld bytes of LDS for this tile", r, span,
             (long long)lds);
  if ((int64_t)sh.cs * (win / 16) > (int64_t)sh.nld * nt)
    SDD_FAIL(SDD_EINVAL, "range %d: delay span %d exceeds this tile's staging capacity", r, span);
  if (span_out) *span_out = span;
  return SDD_OK;
}

// Fraction of (channel pair, neighbouring trial pair) groups of a range
// whose two trials read the same 16-byte words of the staged windows, with
// the matrix-core tiling (DM tiles of dt trials, wavefronts owning trials
// 2w, 2w + 1 of a tile, channels in pairs): the data reads the sharing form
// of the matrix-core kernel skips.
double range_share_fraction(const sdd_plan* p, int32_t r, int32_t dt) {
  const Range& R = p->ranges[r];
  const int32_t ndm = R.ndm(), C = p->nchan;
  // at most about 2^22 groups are looked at: every step-th trial pair
  const int64_t pairs = ndm / 2, per_pair = C / 2;
  const int64_t step = std::max<int64_t>(1, pairs * per_pair >> 22);
  int64_t groups = 0, shared = 0;
  for (int32_t i = 0; i + 1 < ndm; i += (int32_t)(2 * step)) {
    const int32_t i0 = i / dt * dt;
    if (i + 1 >= i0 + dt) continue;
    const int32_t* a = &R.delays[(size_t)i * C];
    const int32_t* b = &R.delays[(size_t)(i + 1) * C];
    const int32_t* z = &R.delays[(size_t)i0 * C];
    for (int32_t c = 0; c + 1 < C; c += 2) {
      const int32_t pa0 = (a[c] - (z[c] & ~15)) & ~15, pb0 = (b[c] - (z[c] & ~15)) & ~15;
      const int32_t pa1 = (a[c + 1] - (z[c + 1] & ~15)) & ~15;
      const int32_t pb1 = (b[c + 1] - (z[c + 1] & ~15)) & ~15;
      shared += (pa0 == pb0 && pa1 == pb1);
      ++groups;
    }
  }
  return groups ? (double)shared / (double)groups : 0.0;
}

sdd_tile default_tile(const sdd_plan* p, int32_t r, int32_t* span_out) {
  // The first LDS shape of the menu that fits (the menu is in preference
  // order), else the direct kernel. Shapes of the sharing matrix-core form
  // (flag 16) come first when at least half of the range's groups share
  // their data reads (fine DM steps), and are skipped otherwise; decimated
  // ranges try the uint16 shapes below first.
  const Range& R = p->ranges[r];
  if (R.dec > 1) {
    // uint16 rows, measured on the decimated ranges of the multi-range plan:
    // the four-copy form with 4 trials per wavefront (23% less time than the
    // two-copy form's 4-channel-stage shape), with 2, then that shape (7-9%
    // faster than its 8-channel stages)
    static const sdd_tile kU16[] = {
        {9, 4, 8, 1, 8, 4}, {9, 2, 8, 1, 8, 4}, {1, 2, 8, 1, 8, 4}};
    for (const sdd_tile& t : kU16) {
      int32_t span = 0;
      if (lds_shape_index(t) >= 0 && check_tile_fits(p, r, t, &span) == SDD_OK) {
        clear_error();  // from the shapes that did not fit
        *span_out = span;
        return t;
      }
    }
  }
  bool share = false;
  for (int k = 0; k < kNumLdsShapes && !share; ++k) {
    const LdsShape& sh = kLdsShapes[k];
    if ((sh.f & 16) != 0)
      share = range_share_fraction(p, r, sh.d * sh.wd) >= kShareThreshold;
  }
  for (int pass = share ? 0 : 1; pass < 2; ++pass)
  for (int k = 0; k < kNumLdsShapes; ++k) {
    const LdsShape& sh = kLdsShapes[k];
    if (((sh.f & 16) != 0) != (pass == 0)) continue;
    sdd_tile t{1 + sh.f, sh.d, sh.wd, sh.wt, 4 * sh.m, sh.cs};
    int32_t span = 0;
    if (check_tile_fits(p, r, t, &span) == SDD_OK) {
      clear_error();  // from the shapes that did not fit
      *span_out = span;
      return t;
    }
  }
  clear_error();
  *span_out = 0;
  return sdd_tile{0, 0, 0, 0, 0, 0};
}

sdd_status plan_geometry(const sdd_plan* p, int64_t nsamp_in, CallGeom* out) {
  CallGeom cg;
  sdd_geometry& g = cg.g;
  std::memset(&g, 0, sizeof(g));
  g.nsamp_in = nsamp_in;
  g.overlap = p->overlap;
  g.n_owned = nsamp_in - p->overlap;
  if (nsamp_in <= 0 || g.n_owned < p->dec_max)
    SDD_FAIL(SDD_EINVAL,
             "nsamp_in %lld too short: needs at least overlap %lld + %d samples",
             (long long)nsamp_in, (long long)p->overlap, p->dec_max);
  const int32_t nw = (int32_t)p->widths.size();
  WsLayout& ws = cg.ws;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  if (p->layout == SDD_TIME_MAJOR) {
    ws.ct_pitch = round_up(nsamp_in, 256);
    ws.ct_off = take(ws.ct_pitch * p->nchan);
  }
  for (const auto& R : p->ranges)
    if (R.dec > 1 && std::find(ws.decs.begin(), ws.decs.end(), R.dec) == ws.decs.end())
      ws.decs.push_back(R.dec);
  std::sort(ws.decs.begin(), ws.decs.end());
  for (int32_t d : ws.decs) {
    int64_t len = nsamp_in / d;
    int64_t pitch = round_up(len, 128);
    ws.dec_len.push_back(len);
    ws.dec_pitch.push_back(pitch);
    ws.dec_off.push_back(take(pitch * 2 * p->nchan));
  }
  int64_t cells_total = 0;
  for (size_t r = 0; r < p->ranges.size(); ++r) {
    const Range& R = p->ranges[r];
    int64_t nr = g.n_owned / R.dec;
    g.n_owned_r[r] = nr;
    g.plane_cols[r] = nr + p->w_max - 1;
    g.ncells[r] = p->cells_for(nr);
    cg.cell_base[r] = cells_total;
    cells_total += g.ncells[r] * R.ndm();
    if (nw > 0) {
      // S2 = sum y^2 < 2^64 with y <= nchan * 255 * dec
      long double ymax = (long double)p->nchan * 255.0L * R.dec;
      if ((long double)nr * ymax * ymax >= 18446744073709551615.0L)
        SDD_FAIL(SDD_ERANGE, "range %zu: %lld owned samples could overflow the 64-bit S2 sum",
                 r, (long long)nr);
    }
  }
  ws.search_cells = cells_total;
  if (nw > 0) {
    ws.cellres_off = take(cells_total * nw * 8);
    ws.moments_off = take((int64_t)p->ndm_total * 16);
    ws.cellbest_off = take(cells_total * 16);
    ws.rowcnt_off = take((int64_t)p->ndm_total * 4);
    ws.rowoff_off = take(((int64_t)p->ndm_total + 1) * 4);
    ws.robust_off = take((int64_t)p->ndm_total * 48);
    if (p->dered_block > 0) {
      for (size_t r = 0; r < p->ranges.size(); ++r)
        ws.dered_nb = std::max<int64_t>(ws.dered_nb,
                                        (g.plane_cols[r] + p->dered_block - 1) / p->dered_block);
      ws.dered_off = take((int64_t)p->ndm_total * ws.dered_nb * 4);
    }
  }
  ws.total = off;
  for (size_t r = 0; r < p->ranges.size(); ++r) {
    ws.plane_pitch[r] = round_up(g.plane_cols[r], 64);
    ws.plane_off[r] = take(ws.plane_pitch[r] * 4 * p->ranges[r].ndm());
  }
  ws.total_planes = off;
  g.workspace_bytes = ws.total;
  g.workspace_bytes_planes = ws.total_planes;
  *out = cg;
  return SDD_OK;
}

sdd_status plan_upload(const sdd_plan* p) {
  std::lock_guard<std::mutex> lk(p->mu);
  if (p->uploaded_device == p->device) return SDD_OK;
  const int32_t C = p->nchan;
  p->d_delays.assign(p->ranges.size(), nullptr);
  for (size_t r = 0; r < p->ranges.size(); ++r) {
    const Range& R = p->ranges[r];
    const int32_t ndm = R.ndm();
    std::vector<int32_t> cm((size_t)ndm * round_up(C, kDelayRowPad), 0);
    for (int32_t i = 0; i < ndm; ++i)
      for (int32_t c = 0; c < C; ++c) cm[(size_t)c * ndm + i] = R.delays[(size_t)i * C + c];
    int32_t* d = nullptr;
    SDD_HIP_TRY(hipMalloc(&d, cm.size() * sizeof(int32_t)));
    p->d_delays[r] = d;
    SDD_HIP_TRY(hipMemcpy(d, cm.data(), cm.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  {
    std::vector<double> all;
    for (const Range& R : p->ranges) all.insert(all.end(), R.dms.begin(), R.dms.end());
    SDD_HIP_TRY(hipMalloc(&p->d_dms, all.size() * sizeof(double)));
    SDD_HIP_TRY(hipMemcpy(p->d_dms, all.data(), all.size() * sizeof(double),
                          hipMemcpyHostToDevice));
  }
  if (!p->widths.empty()) {
    SDD_HIP_TRY(hipMalloc(&p->d_widths, p->widths.size() * sizeof(int32_t)));
    SDD_HIP_TRY(hipMemcpy(p->d_widths, p->widths.data(), p->widths.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
  }
  p->uploaded_device = p->device;
  return SDD_OK;
}

}  // namespace sdd

using namespace sdd;

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

extern "C" sdd_status sdd_plan_create(const sdd_plan_desc* d, sdd_plan** out) {
  clear_error();
  if (!d || !out) SDD_FAIL(SDD_EINVAL, "null descriptor or output pointer");
  *out = nullptr;
  if (!d->freqs_mhz || d->nchan < 1) SDD_FAIL(SDD_EINVAL, "need nchan >= 1 frequencies");
  if (!finite_pos(d->t_samp_s)) SDD_FAIL(SDD_EINVAL, "t_samp must be finite and > 0");
  if ((d->dm_list != nullptr) == (d->ranges != nullptr))
    SDD_FAIL(SDD_EINVAL, "give exactly one of dm_list and ranges");
  if (d->layout != SDD_CHAN_MAJOR && d->layout != SDD_TIME_MAJOR)
    SDD_FAIL(SDD_EINVAL, "unknown layout %d", d->layout);
  if (d->device < 0) SDD_FAIL(SDD_EINVAL, "bad device %d", d->device);
  if (d->nwidths < 0 || d->nwidths > SDD_MAX_WIDTHS)
    SDD_FAIL(SDD_EINVAL, "nwidths must be in [0, %d]", SDD_MAX_WIDTHS);
  if (d->nwidths > 0 && !d->widths) SDD_FAIL(SDD_EINVAL, "null widths");
  if (d->cand_block < 0) SDD_FAIL(SDD_EINVAL, "cand_block must be >= 1 (0 = 1024)");
  if (!std::isfinite(d->threshold)) SDD_FAIL(SDD_EINVAL, "threshold must be finite");

  static std::atomic<uint64_t> next_id{1};
  sdd_plan* p = new sdd_plan();
  p->id = next_id.fetch_add(1);
  p->nchan = d->nchan;
  p->layout = d->layout;
  p->device = d->device;
  p->cand_block = d->cand_block == 0 ? 1024 : d->cand_block;
  p->threshold = d->threshold;
  p->t_samp = d->t_samp_s;
  p->freqs.assign(d->freqs_mhz, d->freqs_mhz + d->nchan);
  for (double f : p->freqs)
    if (!finite_pos(f)) {
      delete p;
      SDD_FAIL(SDD_EINVAL, "frequencies must be finite and > 0");
    }
  for (int32_t k = 0; k < d->nwidths; ++k) {
    int32_t w = d->widths[k];
    if (w < 1 || (k > 0 && w <= d->widths[k - 1])) {
      delete p;
      SDD_FAIL(SDD_EINVAL, "widths must be >= 1 and strictly ascending");
    }
    p->widths.push_back(w);
  }
  p->w_max = p->widths.empty() ? 1 : p->widths.back();
  if (p->w_max > SDD_MAX_WMAX) {
    delete p;
    SDD_FAIL(SDD_EINVAL, "largest width %d exceeds %d", p->w_max, SDD_MAX_WMAX);
  }
  if (d->dm_list) {
    if (d->ndm < 1) {
      delete p;
      SDD_FAIL(SDD_EINVAL, "ndm must be >= 1");
    }
    Range R;
    R.dec = 1;
    R.dms.assign(d->dm_list, d->dm_list + d->ndm);
    p->ranges.push_back(R);
  } else {
    if (d->nranges < 1 || d->nranges > SDD_MAX_RANGES) {
      delete p;
      SDD_FAIL(SDD_EINVAL, "nranges must be in [1, %d]", SDD_MAX_RANGES);
    }
    for (int32_t r = 0; r < d->nranges; ++r) {
      const sdd_dm_range& g = d->ranges[r];
      if (!(g.dm_step > 0.0) || !std::isfinite(g.dm_step) || !std::isfinite(g.dm_lo) ||
          !std::isfinite(g.dm_hi) || g.decimation < 1) {
        delete p;
        SDD_FAIL(SDD_EINVAL, "range %d: need finite lo/hi, step > 0 and decimation >= 1", r);
      }
      double cnt = std::floor((g.dm_hi - g.dm_lo) / g.dm_step + 0.5);
      if (!(cnt >= 1.0) || cnt > 1.0e7) {
        delete p;
        SDD_FAIL(SDD_EINVAL, "range %d: trial count %g out of range", r, cnt);
      }
      Range R;
      R.dec = g.decimation;
      for (int64_t i = 0; i < (int64_t)cnt; ++i) R.dms.push_back(g.dm_lo + (double)i * g.dm_step);
      p->ranges.push_back(R);
    }
  }
  int32_t off = 0;
  for (auto& R : p->ranges) {
    for (double dm : R.dms)
      if (!(dm >= 0.0) || !std::isfinite(dm)) {
        delete p;
        SDD_FAIL(SDD_EINVAL, "trial DMs must be finite and >= 0");
      }
    sdd_status st = build_delays(p->freqs, p->t_samp, R);
    if (st != SDD_OK) {
      delete p;
      return st;
    }
    R.dm_offset = off;
    off += R.ndm();
    p->dec_max = std::max(p->dec_max, R.dec);
  }
  p->ndm_total = off;
  // exact uint32 planes and boxcar sums: nchan * 255 * dec * w_max < 2^32
  long double bmax = (long double)p->nchan * 255.0L * p->dec_max * p->w_max;
  if (bmax >= 4294967296.0L) {
    delete p;
    SDD_FAIL(SDD_ERANGE, "nchan*255*dec*w_max = %.0Lf does not fit 32 bits", bmax);
  }
  int64_t O = 0;
  for (const auto& R : p->ranges)
    O = std::max<int64_t>(O, ((int64_t)R.max_delay + p->w_max - 1) * R.dec);
  p->overlap = O;
  for (size_t r = 0; r < p->ranges.size(); ++r)
    p->ranges[r].tile = default_tile(p, (int32_t)r, &p->ranges[r].tile_span);
  *out = p;
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_destroy(sdd_plan* p) {
  clear_error();
  if (!p) return SDD_OK;
  if (p->uploaded_device >= 0) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->uploaded_device);
    for (int32_t* d : p->d_delays) (void)hipFree(d);
    if (p->d_widths) (void)hipFree(p->d_widths);
    if (p->d_dms) (void)hipFree(p->d_dms);
    (void)hipSetDevice(prev);
  }
  delete p;
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_query(const sdd_plan* p, sdd_plan_info* o) {
  clear_error();
  if (!p || !o) SDD_FAIL(SDD_EINVAL, "null argument");
  std::memset(o, 0, sizeof(*o));
  o->nchan = p->nchan;
  o->nranges = (int32_t)p->ranges.size();
  o->ndm_total = p->ndm_total;
  o->nwidths = (int32_t)p->widths.size();
  o->w_max = p->w_max;
  o->cand_block = p->cand_block;
  o->layout = p->layout;
  o->device = p->device;
  o->overlap = p->overlap;
  for (size_t r = 0; r < p->ranges.size(); ++r) {
    o->ndm[r] = p->ranges[r].ndm();
    o->dm_offset[r] = p->ranges[r].dm_offset;
    o->decimation[r] = p->ranges[r].dec;
    o->max_delay[r] = p->ranges[r].max_delay;
  }
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_delays(const sdd_plan* p, int32_t r, int32_t* host_out) {
  clear_error();
  if (!p || !host_out) SDD_FAIL(SDD_EINVAL, "null argument");
  if (r < 0 || r >= (int32_t)p->ranges.size()) SDD_FAIL(SDD_EINVAL, "bad range %d", r);
  std::memcpy(host_out, p->ranges[r].delays.data(), p->ranges[r].delays.size() * 4);
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_dms(const sdd_plan* p, int32_t r, double* host_out) {
  clear_error();
  if (!p || !host_out) SDD_FAIL(SDD_EINVAL, "null argument");
  if (r < 0 || r >= (int32_t)p->ranges.size()) SDD_FAIL(SDD_EINVAL, "bad range %d", r);
  std::memcpy(host_out, p->ranges[r].dms.data(), p->ranges[r].dms.size() * 8);
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_geometry(const sdd_plan* p, int64_t nsamp_in, sdd_geometry* o) {
  clear_error();
  if (!p || !o) SDD_FAIL(SDD_EINVAL, "null argument");
  CallGeom cg;
  sdd_status st = plan_geometry(p, nsamp_in, &cg);
  if (st != SDD_OK) return st;
  *o = cg.g;
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_get_tile(const sdd_plan* p, int32_t r, sdd_tile* o) {
  clear_error();
  if (!p || !o) SDD_FAIL(SDD_EINVAL, "null argument");
  if (r < 0 || r >= (int32_t)p->ranges.size()) SDD_FAIL(SDD_EINVAL, "bad range %d", r);
  *o = p->ranges[r].tile;
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_set_tile(sdd_plan* p, int32_t r, const sdd_tile* t) {
  clear_error();
  if (!p || !t) SDD_FAIL(SDD_EINVAL, "null argument");
  if (r < -1 || r >= (int32_t)p->ranges.size()) SDD_FAIL(SDD_EINVAL, "bad range %d", r);
  int32_t r0 = r < 0 ? 0 : r, r1 = r < 0 ? (int32_t)p->ranges.size() : r + 1;
  std::vector<int32_t> spans(r1 - r0);
  for (int32_t k = r0; k < r1; ++k) {
    sdd_status st = check_tile_fits(p, k, *t, &spans[k - r0]);
    if (st != SDD_OK) return st;
  }
  for (int32_t k = r0; k < r1; ++k) {
    p->ranges[k].tile = *t;
    p->ranges[k].tile_span = spans[k - r0];
  }
  p->version++;
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_set_stats(sdd_plan* p, int32_t mode, double k, int32_t iters) {
  clear_error();
  if (!p) SDD_FAIL(SDD_EINVAL, "null plan");
  if (mode != SDD_STATS_MOMENTS && mode != SDD_STATS_CLIPPED && mode != SDD_STATS_MEDIAN_MAD)
    SDD_FAIL(SDD_EINVAL, "unknown statistics mode %d", mode);
  if (mode == SDD_STATS_CLIPPED && (!(k > 0.0) || !std::isfinite(k) || iters < 1 || iters > 64))
    SDD_FAIL(SDD_EINVAL, "clipping needs k > 0 and 1..64 iterations");
  p->stats_mode = mode;
  if (mode == SDD_STATS_CLIPPED) {
    p->clip_k = k;
    p->clip_iters = iters;
  }
  p->version++;  // cached batch graphs hold the old search arguments
  return SDD_OK;
}

extern "C" sdd_status sdd_plan_set_dereddening(sdd_plan* p, int32_t block, int32_t half) {
  clear_error();
  if (!p) SDD_FAIL(SDD_EINVAL, "null plan");
  if (block == 0) {
    p->dered_block = p->dered_half = 0;
    p->version++;
    return SDD_OK;
  }
  if (p->widths.empty()) SDD_FAIL(SDD_EINVAL, "de-reddening needs a plan with boxcar widths");
  if (block < 64 || block > 4096 || (block & (block - 1)) != 0)
    SDD_FAIL(SDD_EINVAL, "block %d is not a power of two in 64..4096", block);
  if (half < 1 || (int64_t)(2 * half + 1) * block > 4096)
    SDD_FAIL(SDD_EINVAL, "window (2*%d+1)*%d must hold 1..4096 samples with half >= 1", half,
             block);
  if ((int64_t)(2 * half + 1) * block <= 2 * (int64_t)p->w_max)
    SDD_FAIL(SDD_EINVAL, "window (2*%d+1)*%d must exceed twice the widest boxcar (%d)", half,
             block, p->w_max);
  if ((int64_t)p->nchan * 255 * p->dec_max >= ((int64_t)1 << 30))
    SDD_FAIL(SDD_ERANGE, "full scale nchan*255*dec_max exceeds 2^30");
  p->dered_block = block;
  p->dered_half = half;
  p->version++;  // cached batch graphs hold the old search arguments
  return SDD_OK;
}

extern "C" sdd_status sdd_tile_menu(sdd_tile* host_out, int32_t max, int32_t* n_out) {
  clear_error();
  if (!n_out || (max > 0 && !host_out)) SDD_FAIL(SDD_EINVAL, "null argument");
  const auto& m = tile_menu();
  *n_out = (int32_t)m.size();
  for (int32_t k = 0; k < max && k < (int32_t)m.size(); ++k) host_out[k] = m[k];
  return SDD_OK;
}
