// Internal declarations of libspotdd: the plan, the workspace layout and the
// kernel launchers. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "spotdd.h"

namespace sdd {

// Records the message returned by sdd_last_error() on this thread.
void set_error(const char* fmt, ...);
void clear_error();

#define SDD_HIP_TRY(expr)                                                        \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::sdd::set_error("%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                \
      return SDD_EDEVICE;                                                        \
    }                                                                            \
  } while (0)

#define SDD_FAIL(code, ...)          \
  do {                               \
    ::sdd::set_error(__VA_ARGS__);   \
    return code;                     \
  } while (0)

// Workspaces hold 64-bit atomics and 128-bit vectors at 256-byte offsets.
#define SDD_CHECK_WS_ALIGN(ws)                                                   \
  do {                                                                           \
    if ((ws) && reinterpret_cast<uintptr_t>(ws) % 256 != 0)                      \
      SDD_FAIL(SDD_EINVAL, "the workspace must be 256-byte aligned");           \
  } while (0)

constexpr double kDispersionConstant = 4.148808e3;  // s MHz^2 pc^-1 cm^3
// Device delay tables are padded with zero rows to a multiple of this many
// channels, so a kernel stage of up to this many channels reads them unmasked.
constexpr int32_t kDelayRowPad = 16;

// Brackets one stage's launches with HIP events on its stream while timing is
// enabled (sdd_profile_enable); does nothing otherwise.
class StageTimer {
 public:
  StageTimer(int stage, hipStream_t s);
  ~StageTimer();
  StageTimer(const StageTimer&) = delete;
  StageTimer& operator=(const StageTimer&) = delete;

 private:
  int stage_;
  hipStream_t s_;
  hipEvent_t a_{}, b_{};
  bool active_ = false;
};

struct Range {
  int32_t dec = 1;
  std::vector<double> dms;
  std::vector<int32_t> delays;  // host, [ndm][nchan]
  int32_t max_delay = 0;
  int32_t dm_offset = 0;
  sdd_tile tile{};
  int32_t tile_span = 0;  // largest delay difference inside one DM tile of `tile`
  int32_t ndm() const { return (int32_t)dms.size(); }
};

// Offsets (bytes) of every region of the per-call workspace.
struct WsLayout {
  int64_t ct_off = -1, ct_pitch = 0;            // corner-turned input [C][ct_pitch] u8
  std::vector<int32_t> decs;                     // distinct decimations > 1, ascending
  std::vector<int64_t> dec_off, dec_pitch, dec_len;  // u16 [C][pitch] each
  int64_t plane_off[SDD_MAX_RANGES] = {0};       // library planes (with_planes only)
  int64_t plane_pitch[SDD_MAX_RANGES] = {0};     // elements
  int64_t cellres_off = 0;   // [sum_r ndm_r * ncells_r * nw] u64 (B << 32) | ~(j - cell start)
  int64_t moments_off = 0;   // [ndm_total] {u64 s1, u64 s2}
  int64_t cellbest_off = 0;  // [sum_r ndm_r * ncells_r] {f64 snr, i32 j, i32 w}
  int64_t rowcnt_off = 0;    // [ndm_total] i32
  int64_t rowoff_off = 0;    // [ndm_total + 1] i32
  int64_t robust_off = 0;    // [ndm_total] {f64 mu, f64 sigma, u64 cnt, s1, s2, pad}
  int64_t dered_off = 0;     // [ndm_total][dered_nb] u32 (de-reddening only)
  int64_t dered_nb = 0;
  int64_t search_cells = 0;  // sum_r ndm_r * ncells_r
  int64_t total = 0;         // bytes without library planes
  int64_t total_planes = 0;  // bytes with library planes
};

// Per-call geometry derived from nsamp_in (see spotdd.h, "extent").
struct CallGeom {
  sdd_geometry g{};
  WsLayout ws;
  int64_t cell_base[SDD_MAX_RANGES] = {0};  // first global cell of range r
};

}  // namespace sdd

struct sdd_plan {
  int32_t nchan = 0, layout = 0, device = 0, cand_block = 1024;
  float threshold = 0.f;
  double t_samp = 0.0;
  std::vector<double> freqs;
  std::vector<int32_t> widths;
  int32_t w_max = 1;
  std::vector<sdd::Range> ranges;
  int64_t overlap = 0;
  int32_t ndm_total = 0;
  int32_t dec_max = 1;
  // noise estimate of the search's S/N (sdd_plan_set_stats)
  int32_t stats_mode = 0;
  double clip_k = 3.0;
  int32_t clip_iters = 3;
  // running-median de-reddening of the searched series (sdd_plan_set_dereddening)
  int32_t dered_block = 0;  // D (0: off)
  int32_t dered_half = 0;   // h

  uint64_t id = 0;       // process-unique, never reused
  uint64_t version = 0;  // bumped whenever the tile choice changes

  // device copies, made on first use
  mutable std::mutex mu;
  mutable int uploaded_device = -1;
  // per range, [round_up(nchan, kDelayRowPad)][ndm_r]; rows past nchan are 0
  mutable std::vector<int32_t*> d_delays;
  mutable int32_t* d_widths = nullptr;
  mutable double* d_dms = nullptr;  // every trial DM, ranges in order (global trial index)

  int32_t cells_for(int64_t n_owned_r) const {
    return widths.empty() ? 0 : (int32_t)((n_owned_r + cand_block - 1) / cand_block);
  }
};

namespace sdd {

sdd_status plan_geometry(const sdd_plan* p, int64_t nsamp_in, CallGeom* out);
sdd_status plan_upload(const sdd_plan* p);
bool tile_in_menu(const sdd_tile& t);
const std::vector<sdd_tile>& tile_menu();
// Largest delay difference across any DM tile of dm_tile consecutive trials of
// range r, over all channels (LDS window sizing).
int32_t range_span(const sdd_plan* p, int32_t r, int32_t dm_tile);
// Checks that tile t can run range r; on success *span_out (if given) receives
// the DM-tile delay span the kernel's LDS window must cover.
sdd_status check_tile_fits(const sdd_plan* p, int32_t r, const sdd_tile& t,
                           int32_t* span_out = nullptr);
sdd_tile default_tile(const sdd_plan* p, int32_t r, int32_t* span_out);
// LDS window bytes per copy for a tile of tt samples of es bytes and the
// given delay span (samples).
inline int32_t lds_window_bytes(int32_t tt, int32_t span, int es) {
  return (es * (tt + span + 32) + 15) / 16 * 16;
}

// ---- kernel launchers (k_*.hip) ----------------------------------------

// ring_rows > 0: `in` is a ring of ring_rows spectra and the window starts at
// row ring_start (rows wrap modulo ring_rows).
// lut (optional, [nchan][256]) maps every byte of channel c through
// lut[c][v]; tmask (optional, [nsamp]) zeroes window sample t where tmask[t]
// is 0 (RFI pre-conditioning).
hipError_t launch_corner_turn(const uint8_t* in, int64_t nsamp, int64_t in_pitch, int32_t nchan,
                              uint8_t* out, int64_t out_pitch, hipStream_t s,
                              int64_t ring_rows = 0, int64_t ring_start = 0,
                              const uint8_t* lut = nullptr, const uint8_t* tmask = nullptr);
// Channel rows copied through the same lut / tmask.
hipError_t launch_precond_rows(const uint8_t* in, int64_t in_pitch, int64_t nsamp, int32_t nchan,
                               const uint8_t* lut, const uint8_t* tmask, uint8_t* out,
                               int64_t out_pitch, hipStream_t s);
// out[c][j] = sum_{k<factor} in[c][j*factor+k], j < out_len; in is u8 or u16.
// Power-of-two decimation levels 2, 4, 8, 16 (index 0..3) built in one pass
// from uint8 rows; out[l] == nullptr skips level l.
struct DecLevels {
  uint16_t* out[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t pitch[4] = {0, 0, 0, 0};  // elements
  int64_t len[4] = {0, 0, 0, 0};    // outputs per row
  int vec[4] = {0, 0, 0, 0};        // set by the launcher: aligned vector stores
};
hipError_t launch_decimate_pow2(const uint8_t* in, int64_t in_pitch, int64_t nsamp, int32_t nchan,
                                const DecLevels& lv, hipStream_t s);
hipError_t launch_decimate(const void* in, int in_bytes, int64_t in_pitch, int32_t nchan,
                           int32_t factor, uint16_t* out, int64_t out_pitch, int64_t out_len,
                           hipStream_t s);

struct DedispArgs {
  const void* x;          // channel rows of the range's input (u8 or u16)
  int32_t elem_bytes;     // 1 or 2
  int64_t x_pitch;        // elements between channel rows
  int64_t x_len;          // valid samples per row
  int32_t nchan;
  const int32_t* delays;  // device [nchan][ndm]
  int32_t ndm;
  uint32_t* plane;
  int64_t plane_pitch;    // elements
  int64_t cols;           // columns to produce
  int32_t max_val;        // largest input value (255 * dec)
  sdd_tile tile;
  int32_t span;           // largest delay difference over a DM tile of the chosen shape
  int32_t max_delay;      // largest delay of the range (samples of x)
};
hipError_t launch_dedisperse(const DedispArgs& a, hipStream_t s);

struct SearchRange {
  const uint32_t* plane;
  int64_t pitch;
  int64_t n_owned;     // N_r
  int32_t ndm;
  int32_t dm_offset;   // global trial index of row 0
  int32_t ncells;
  int32_t full_scale;  // M = nchan * 255 * dec, bound of every plane sample
  int64_t cell_base;   // global cell index of (row 0, cell 0)
};
struct SearchArgs {
  SearchRange r[SDD_MAX_RANGES];
  int32_t nranges;
  int32_t ndm_total;
  int32_t nwidths;
  int32_t w_max;
  int32_t widths[SDD_MAX_WIDTHS];
  int32_t cand_block;
  float threshold;
  int32_t max_cells;     // max_r ncells_r
  int32_t cap;
  int64_t max_boxcar;    // bound on any boxcar sum: nchan * 255 * dec_max * w_max
  int64_t max_sample;    // bound on any plane value: nchan * 255 * dec_max
  int32_t stats_mode;    // SDD_STATS_*
  int32_t clip_iters;
  double clip_k;
  int64_t robust_off;
  int32_t dered_shift;   // log2 of the de-reddening block D; 0: off
  int32_t dered_half;    // h: the median window is blocks k-h..k+h
  int32_t dered_elems;   // samples per lane of k_dered_base's window (template)
  int32_t dered_nb;      // baselines per trial in the workspace
  int64_t dered_off;     // [ndm_total][dered_nb] u32 block baselines
  uint8_t* ws;           // workspace base
  int64_t cellres_off, moments_off, cellbest_off, rowcnt_off, rowoff_off;
  sdd_dm_best* best;
  sdd_dm_stats* stats;   // may be null
  sdd_candidate* cands;  // may be null when cap == 0
  int32_t* ncand;
};
hipError_t launch_search(const SearchArgs& a, hipStream_t s);

// ---- one chunk's launch sequence (capi.cpp) -------------------------------

// Corner turn and decimations of one chunk; appends one dedispersion job per
// DM range (not launched).
// RFI pre-conditioning of a call's input: x'[c][t] = tmask[t] ? lut[c][x] : 0
// (either map may be null). Channel-major input is copied through it into
// rows [nchan][rows_pitch] (scratch past the call's workspace).
struct Precond {
  const uint8_t* lut = nullptr;
  const uint8_t* tmask = nullptr;
  uint8_t* rows = nullptr;
  int64_t rows_pitch = 0;
};
sdd_status prep_item(const sdd_plan* p, const CallGeom& cg, const uint8_t* d_in, int64_t nsamp_in,
                     int64_t in_pitch, uint32_t* const* planes, const int64_t* pitch, uint8_t* ws,
                     hipStream_t s, std::vector<DedispArgs>* jobs, int64_t ring_rows = 0,
                     int64_t ring_start = 0, const Precond* pre = nullptr);
sdd_status run_dedisperse(const sdd_plan* p, const CallGeom& cg, const uint8_t* d_in,
                          int64_t nsamp_in, int64_t in_pitch, uint32_t* const* planes,
                          const int64_t* pitch, uint8_t* ws, hipStream_t s,
                          const Precond* pre = nullptr);
sdd_status run_search(const sdd_plan* p, const CallGeom& cg, const uint32_t* const* planes,
                      const int64_t* pitch, sdd_dm_best* best, sdd_dm_stats* stats,
                      sdd_candidate* cands, int32_t cap, int32_t* ncand, uint8_t* ws,
                      hipStream_t s);
sdd_status check_input(const sdd_plan* p, const uint8_t* d_in, int64_t nsamp_in, int64_t in_pitch);
sdd_status check_planes(const sdd_plan* p, const CallGeom& cg, const void* const* planes,
                        const int64_t* pitch);
// Dedispersion of a set of jobs: jobs sharing an LDS tile shape go through the
// persistent multi-job kernel; the rest are launched one by one.
// Tile counters a batch workspace holds for its persistent launches (8 per
// launch: one per XCD).
constexpr int32_t kBatchTickets = 64;
sdd_status launch_jobs_persistent(const std::vector<DedispArgs>& jobs, uint32_t* tickets,
                                  hipStream_t s);

// ---- batches (batch.cpp) ------------------------------------------------


// One chunk of a batch; ring_rows > 0 marks a time-major ring input whose
// window starts at row ring_start.
struct BatchJob {
  sdd_batch_item it;
  int64_t ring_rows = 0, ring_start = 0;
};
struct ItemGeom {
  CallGeom cg;
  int64_t ws_off = 0, ws_bytes = 0;
  uint32_t* planes[SDD_MAX_RANGES];
  int64_t pitch[SDD_MAX_RANGES];
};
sdd_status batch_layout(const BatchJob* items, int32_t n, std::vector<ItemGeom>* out,
                        int64_t* total);
int64_t batch_tickets_off(const std::vector<ItemGeom>& geo);
sdd_status enqueue_batch(const BatchJob* items, int32_t n, int32_t flags,
                         std::vector<ItemGeom>& geo, uint8_t* ws, hipStream_t s);

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace sdd
