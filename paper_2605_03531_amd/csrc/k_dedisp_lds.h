// Arguments and shape menu of the LDS-tiled dedispersion kernel.
#pragma once

#include "sdd_internal.h"

namespace sdd {

struct LdsArgs {
  const uint8_t* x;       // channel rows (uint8, or uint16 when es == 2)
  int64_t x_pitch;        // elements between rows
  int64_t x_len;          // valid samples per row
  int32_t nchan;
  int32_t ndm;
  const int32_t* delays;  // device [nchan][ndm]
  uint32_t* plane;
  int64_t plane_pitch;
  int64_t cols;
  int32_t win;            // LDS window bytes per copy (multiple of 16)
  int32_t n_dtiles, n_ttiles;
  int32_t aligned;        // rows start 16-byte aligned
  int32_t es;             // element bytes: 1 or 2
  int32_t flush;          // channels per 16-bit flush (es == 2; multiple of the stage)
  int32_t n_tt_interior;  // time tiles [0, n) whose staging loads all lie inside the rows
};


// Compile-time shape of one instantiation.
struct LdsShape {
  int d;      // trials per wavefront
  int m;      // 512-sample chunks per lane group
  int wd;     // wavefronts along DM
  int wt;     // wavefronts along time
  int cs;     // channels per LDS stage
  int nld;    // 16-byte staging loads per thread per stage
  int f;      // variant flags: 2 = third word through a 64-bit read,
              // 4 = matrix-core form (uint8 rows), 4 | 16 = matrix-core form
              // that skips the data reads neighbouring trials share,
              // 8 = vector form with four shifted copies per window (uint16
              // rows)
};

// Samples one tile of a shape covers for elements of es bytes.
inline int32_t lds_tile_samples(const LdsShape& sh, int es) { return 512 / es * sh.m * sh.wt; }
// Channels a range of element maximum max_val may add into 16-bit fields
// before a flush, rounded down to a multiple of the stage (0: not possible).
inline int32_t lds_flush_period(const LdsShape& sh, int32_t max_val) {
  const int32_t f = 65535 / max_val;
  return f >= 256 ? 256 : (f / sh.cs) * sh.cs;
}

// LDS bytes of one workgroup for windows of win bytes (the kernel's own
// sizing: two stage buffers of cs windows, two copies of each in the vector
// form, four with flag 8; one copy and a 1 KiB selection table in the
// matrix-core form).
inline int64_t lds_tile_bytes(const LdsShape& sh, int64_t win) {
  if ((sh.f & 4) != 0) return 2 * (int64_t)sh.cs * win + 1024;
  return 2 * (int64_t)sh.cs * ((sh.f & 8) != 0 ? 4 : 2) * win;
}
// Whether a shape's form takes rows of es-byte elements.
inline bool lds_shape_takes(const LdsShape& sh, int es) {
  if ((sh.f & 4) != 0) return es == 1;
  if ((sh.f & 8) != 0) return es == 2;
  return es == 1 || es == 2;
}

// Sharing matrix-core shapes (flag 16) are the default for a range when at
// least this fraction of its (channel pair, trial pair) groups read the same
// data words for both trials.
constexpr double kShareThreshold = 0.5;

extern const LdsShape kLdsShapes[];
extern const int kNumLdsShapes;

// Jobs of one persistent launch (kernel argument, so at most kMaxJobs).
constexpr int kMaxJobs = 32;
struct MultiArgs {
  LdsArgs jobs[kMaxJobs];
  int32_t tile_base[kMaxJobs + 1];  // first global tile of each job; [njobs] = total
  int32_t njobs;
  uint32_t* tickets;                // 8 zeroed counters, one per XCD
};

hipError_t launch_dedisperse_lds(const LdsArgs& a, int shape, hipStream_t s);
// LDS-kernel arguments of one job; returns its shape index, or -1 when the
// job must take the direct kernel (decimated input, unaligned plane, ...).
int lds_args_for(const DedispArgs& a, LdsArgs* out);
// All jobs must fit the shape; max_win = largest job window.
hipError_t launch_dedisperse_lds_multi(const MultiArgs& m, int32_t max_win, int shape,
                                       hipStream_t s);

}  // namespace sdd
