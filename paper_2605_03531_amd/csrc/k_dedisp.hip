// Brute-force incoherent dedispersion kernels (Section 3.2: every trial DM
// sums all channels along its delay curve; Section 2.1: many trial DMs).
//   plane[i][j] = sum_c x[c][j + delay[c][i]],  j < cols   (exact uint32)
#include <algorithm>

#include "k_dedisp_lds.h"
#include "sdd_internal.h"

namespace sdd {
int lds_shape_index(const sdd_tile& t);
namespace {

// Direct kernel: one thread per (trial, 4 consecutive columns), a plain
// channel loop reading the input straight from global memory. It is the
// simplest correct form and the fallback for shapes the tiled kernel does
// not take.
template <typename Tin>
__global__ __launch_bounds__(256) void k_dedisp_direct(const Tin* __restrict__ x, int64_t xp,
                                                       int32_t nchan,
                                                       const int32_t* __restrict__ dcm,
                                                       int32_t ndm, uint32_t* __restrict__ plane,
                                                       int64_t pp, int64_t cols) {
  const int32_t i = blockIdx.x;
  const int64_t j0 = ((int64_t)blockIdx.y * blockDim.x + threadIdx.x) * 4;
  if (j0 >= cols) return;
  const int nv = cols - j0 < 4 ? (int)(cols - j0) : 4;
  uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  if (nv == 4) {
    for (int32_t c = 0; c < nchan; ++c) {
      const Tin* r = x + (int64_t)c * xp + j0 + dcm[(int64_t)c * ndm + i];
      a0 += r[0];
      a1 += r[1];
      a2 += r[2];
      a3 += r[3];
    }
  } else {
    for (int32_t c = 0; c < nchan; ++c) {
      const Tin* r = x + (int64_t)c * xp + j0 + dcm[(int64_t)c * ndm + i];
      a0 += r[0];
      if (nv > 1) a1 += r[1];
      if (nv > 2) a2 += r[2];
    }
  }
  uint32_t* o = plane + (int64_t)i * pp + j0;
  o[0] = a0;
  if (nv > 1) o[1] = a1;
  if (nv > 2) o[2] = a2;
  if (nv > 3) o[3] = a3;
}

}  // namespace

int lds_args_for(const DedispArgs& a, LdsArgs* out) {
  const int shape = lds_shape_index(a.tile);
  const bool plane_ok = ((uintptr_t)a.plane % 16 == 0) && (a.plane_pitch % 4 == 0);
  if (shape < 0 || !plane_ok || a.cols <= 0 || a.ndm <= 0) return -1;
  const LdsShape& sh = kLdsShapes[shape];
  const int es = a.elem_bytes;
  const int32_t flush = lds_flush_period(sh, a.max_val);
  if (es < 1 || es > 2 || flush < sh.cs) return -1;
  if (!lds_shape_takes(sh, es)) return -1;
  LdsArgs& l = *out;
  l = LdsArgs{};
  l.x = (const uint8_t*)a.x;
  l.x_pitch = a.x_pitch;
  l.x_len = a.x_len;
  l.nchan = a.nchan;
  l.ndm = a.ndm;
  l.delays = a.delays;
  l.plane = a.plane;
  l.plane_pitch = a.plane_pitch;
  l.cols = a.cols;
  const int32_t tt = lds_tile_samples(sh, es), dt = sh.d * sh.wd;
  l.win = lds_window_bytes(tt, a.span, es);
  l.n_dtiles = (a.ndm + dt - 1) / dt;
  l.n_ttiles = (int32_t)((a.cols + tt - 1) / tt);
  l.aligned = ((uintptr_t)a.x % 16 == 0) && ((a.x_pitch * es) % 16 == 0);
  l.es = es;
  l.flush = flush;
  // the kernel forms row offsets of one stage in 32 bits
  const int64_t stage_bytes = (int64_t)sh.cs * a.x_pitch * es + l.win + 32 + (int64_t)es * a.max_delay;
  if (stage_bytes >= ((int64_t)1 << 32)) return -1;
  // tile t is interior when its last staging byte, es*(t*tt + max_delay) +
  // win + 4 (+ 8 with four copies), is inside the row
  const int64_t room =
      (int64_t)es * (a.x_len - a.max_delay) - l.win - ((sh.f & 8) != 0 ? 8 : 4);
  int64_t n_int = 0;
  if (l.aligned && room >= 0) n_int = room / ((int64_t)es * tt) + 1;
  l.n_tt_interior = (int32_t)std::min<int64_t>(n_int, l.n_ttiles);
  return shape;
}

hipError_t launch_dedisperse(const DedispArgs& a, hipStream_t s) {
  if (a.cols <= 0 || a.ndm <= 0) return hipSuccess;
  LdsArgs lds_args;
  const int shape = lds_args_for(a, &lds_args);
  if (shape >= 0) return launch_dedisperse_lds(lds_args, shape, s);
  const int64_t per_block = 256 * 4;
  const int64_t nyb = (a.cols + per_block - 1) / per_block;
  if (nyb > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)a.ndm, (unsigned)nyb);
  if (a.elem_bytes == 1)
    hipLaunchKernelGGL(k_dedisp_direct<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)a.x,
                       a.x_pitch, a.nchan, a.delays, a.ndm, a.plane, a.plane_pitch, a.cols);
  else
    hipLaunchKernelGGL(k_dedisp_direct<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)a.x,
                       a.x_pitch, a.nchan, a.delays, a.ndm, a.plane, a.plane_pitch, a.cols);
  return hipGetLastError();
}

}  // namespace sdd
