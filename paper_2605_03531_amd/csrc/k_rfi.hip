// RFI pre-conditioning of one chunk before dedispersion (Section 2.1 and
// the paper's figure of its RFI tool): the average spectrum (mean of each
// channel), its moving median over a window of channels as the bandpass,
// channels that are robust-sigma outliers of the bandpass-corrected
// spectrum flagged, the zero-DM series over the unflagged channels, its
// outlier samples flagged, the two flaggings repeated; then exact integer
// maps (a per-channel byte table and a time mask) that the corner turn (or a
// row copy) applies before dedispersion.
//
// Medians are exact selections: a single workgroup finds the k-th smallest
// of n 64-bit keys (FP64 values mapped to order-preserving integers) by one
// 256-bin histogram pass per byte, most significant first. All arithmetic is
// FP64 or exact integer, in the order of the stated definitions.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sdd_internal.h"

namespace sdd {
namespace {

constexpr double kMadScale = 1.4826;
constexpr int kMaxWindow = 63;

__device__ __host__ inline uint64_t f64_key(double v) {
  uint64_t b;
  memcpy(&b, &v, 8);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __host__ inline double key_f64(uint64_t k) {
  const uint64_t b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
  double v;
  memcpy(&v, &b, 8);
  return v;
}

struct RfiArgs {
  const uint8_t* rows;  // [C][pitch] channel rows
  int64_t pitch;
  int32_t C;
  int64_t T;
  int32_t window;
  double k_chan, k_time;
  // workspace
  double* m;          // [C] channel means
  double* b;          // [C] bandpass
  double* r;          // [C] residual spectrum
  int32_t* cflag;     // [C]
  int64_t* z;         // [T] zero-DM series
  int32_t* tflag;     // [T]
  uint8_t* keep8;     // [T] 0xff for an unflagged sample, 0 for a flagged one
  uint64_t* keys;     // [max(C, T)] selection keys
  uint64_t* sel;      // [8] selection results
  int64_t* nt;        // [1] unflagged samples
};

// ---- k-th smallest of n keys (one workgroup of 1024) ----
__global__ __launch_bounds__(1024) void k_select(const uint64_t* keys, int64_t n, int64_t k,
                                                 int top_byte, uint64_t* out) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ int64_t s_k;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_prefix = 0;
    s_k = k;
  }
  __syncthreads();
  uint64_t hmask = 0;  // bytes above the current one, already decided
  for (int byte = top_byte; byte >= 0; --byte) {
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    const uint64_t prefix = s_prefix;
    const int sh = 8 * byte;
    for (int64_t i = tid; i < n; i += 1024) {
      const uint64_t v = keys[i];
      if ((v & hmask) == prefix) atomicAdd(&hist[(v >> sh) & 255u], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      int64_t kk = s_k;
      int bin = 0;
      for (; bin < 255; ++bin) {
        if (kk < (int64_t)hist[bin]) break;
        kk -= hist[bin];
      }
      s_k = kk;
      s_prefix = prefix | ((uint64_t)bin << sh);
    }
    __syncthreads();
    hmask |= (uint64_t)255 << sh;
  }
  if (tid == 0) *out = s_prefix;
}

__global__ __launch_bounds__(256) void k_clear_tflag(RfiArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < a.T) {
    a.tflag[t] = 0;
    a.keep8[t] = 0xff;
  }
}

// Sum of the 4 bytes of w (SWAR: two 16-bit fields, then their sum).
__device__ inline uint32_t byte_sum4(uint32_t w) {
  const uint32_t e = (w & 0x00ff00ffu) + ((w >> 8) & 0x00ff00ffu);
  return (e & 0xffffu) + (e >> 16);
}

// ---- unflagged sample count ----
__global__ __launch_bounds__(1024) void k_count_keep(RfiArgs a) {
  __shared__ unsigned long long part[16];
  const int tid = threadIdx.x;
  unsigned long long c = 0;
  for (int64_t t = tid; t < a.T; t += 1024) c += a.tflag[t] ? 0 : 1;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((tid & 63) == 0) part[tid >> 6] = c;
  __syncthreads();
  if (tid == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < 16; ++w) s += part[w];
    *a.nt = (int64_t)s;
  }
}

// ---- channel means over unflagged samples (all when none is unflagged) ----
// VEC: rows 16-byte aligned: 16 samples per load, masked with keep8.
template <bool VEC>
__global__ __launch_bounds__(256) void k_chan_mean(RfiArgs a) {
  __shared__ unsigned long long part[4];
  const int32_t c = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t nt = *a.nt;
  const bool all = nt == 0;
  const uint8_t* row = a.rows + (int64_t)c * a.pitch;
  unsigned long long s = 0;
  int64_t t0 = 0;
  if constexpr (VEC) {
    const int64_t nv = a.T / 16;
    const uint32_t any = all ? 0xffffffffu : 0u;
    for (int64_t v = tid; v < nv; v += 256) {
      const uint4 x = reinterpret_cast<const uint4*>(row)[v];
      const uint4 k = reinterpret_cast<const uint4*>(a.keep8)[v];
      s += byte_sum4(x.x & (k.x | any)) + byte_sum4(x.y & (k.y | any)) +
           byte_sum4(x.z & (k.z | any)) + byte_sum4(x.w & (k.w | any));
    }
    t0 = nv * 16;
  }
  for (int64_t t = t0 + tid; t < a.T; t += 256)
    if (all || !a.tflag[t]) s += row[t];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((tid & 63) == 0) part[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    const unsigned long long tot = part[0] + part[1] + part[2] + part[3];
    a.m[c] = (double)tot / (double)(all ? a.T : nt);
  }
}

// ---- moving lower median of the spectrum, residual, keys ----
__global__ __launch_bounds__(256) void k_bandpass(RfiArgs a) {
  const int32_t c = blockIdx.x * 256 + threadIdx.x;
  if (c >= a.C) return;
  const int h = a.window / 2;
  const int32_t lo = c - h < 0 ? 0 : c - h;
  const int32_t hi = c + h + 1 > a.C ? a.C : c + h + 1;
  double w[kMaxWindow];
  int n = 0;
  for (int32_t q = lo; q < hi; ++q) {
    // insertion into the sorted prefix
    const double v = a.m[q];
    int j = n++;
    while (j > 0 && w[j - 1] > v) {
      w[j] = w[j - 1];
      --j;
    }
    w[j] = v;
  }
  const double bc = w[(n - 1) / 2];
  a.b[c] = bc;
  a.r[c] = a.m[c] - bc;
  a.keys[c] = f64_key(a.m[c] - bc);
}

__global__ __launch_bounds__(256) void k_absdev_f64(RfiArgs a, const double* v, int32_t n,
                                                    const uint64_t* med) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  a.keys[i] = f64_key(fabs(v[i] - key_f64(*med)));
}

__global__ __launch_bounds__(256) void k_cflag(RfiArgs a) {
  const int32_t c = blockIdx.x * 256 + threadIdx.x;
  if (c >= a.C) return;
  const double med = key_f64(a.sel[0]);
  const double sig = kMadScale * key_f64(a.sel[1]);
  a.cflag[c] = (sig > 0.0 && fabs(a.r[c] - med) > a.k_chan * sig) ? 1 : 0;
}

// ---- zero-DM series over unflagged channels ----
// Zero-DM series: blockIdx.y takes channels [64 y, 64 y + 64); each thread 4
// consecutive samples (one 32-bit load per channel when VEC: rows 4-byte
// aligned), added into z with integer atomics (z cleared first).
template <bool VEC>
__global__ __launch_bounds__(256) void k_zero_dm(RfiArgs a) {
  const int64_t t = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (t >= a.T) return;
  const int32_t c0 = blockIdx.y * 64, c1 = min(c0 + 64, a.C);
  uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  if (VEC && t + 4 <= a.T) {
    for (int32_t c = c0; c < c1; ++c) {
      if (a.cflag[c]) continue;
      const uint32_t w = *reinterpret_cast<const uint32_t*>(a.rows + (int64_t)c * a.pitch + t);
      s0 += w & 255u;
      s1 += (w >> 8) & 255u;
      s2 += (w >> 16) & 255u;
      s3 += w >> 24;
    }
  } else {
    for (int32_t c = c0; c < c1; ++c) {
      if (a.cflag[c]) continue;
      const uint8_t* r = a.rows + (int64_t)c * a.pitch + t;
      s0 += r[0];
      if (t + 1 < a.T) s1 += r[1];
      if (t + 2 < a.T) s2 += r[2];
      if (t + 3 < a.T) s3 += r[3];
    }
  }
  unsigned long long* z = reinterpret_cast<unsigned long long*>(a.z);
  atomicAdd(&z[t], (unsigned long long)s0);
  if (t + 1 < a.T) atomicAdd(&z[t + 1], (unsigned long long)s1);
  if (t + 2 < a.T) atomicAdd(&z[t + 2], (unsigned long long)s2);
  if (t + 3 < a.T) atomicAdd(&z[t + 3], (unsigned long long)s3);
}

__global__ __launch_bounds__(256) void k_clear_z(RfiArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < a.T) a.z[t] = 0;
}

__global__ __launch_bounds__(256) void k_z_keys(RfiArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < a.T) a.keys[t] = (uint64_t)a.z[t];
}

__global__ __launch_bounds__(256) void k_absdev_i64(RfiArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.T) return;
  const int64_t d = a.z[t] - (int64_t)a.sel[2];
  a.keys[t] = (uint64_t)(d < 0 ? -d : d);
}

__global__ __launch_bounds__(256) void k_tflag(RfiArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.T) return;
  const int64_t med = (int64_t)a.sel[2];
  const double sig = kMadScale * (double)(int64_t)a.sel[3];
  const int64_t d = a.z[t] - med;
  const bool flag = sig > 0.0 && (double)(d < 0 ? -d : d) > a.k_time * sig;
  a.tflag[t] = flag ? 1 : 0;
  a.keep8[t] = flag ? 0 : 0xff;
}

__global__ __launch_bounds__(256) void k_bp_keys(RfiArgs a) {
  const int32_t c = blockIdx.x * 256 + threadIdx.x;
  if (c < a.C) a.keys[c] = f64_key(a.b[c]);
}

// lut[c][v] = flagged ? 0 : clip(v - floor(b_c + 0.5) + floor(median(b) + 0.5), 0, 255)
__global__ __launch_bounds__(256) void k_emit_lut(RfiArgs a, uint8_t* lut, int32_t* chan_flags) {
  const int32_t c = blockIdx.x;
  const int v = threadIdx.x;
  const int64_t B = (int64_t)floor(a.b[c] + 0.5);
  const int64_t L = (int64_t)floor(key_f64(a.sel[4]) + 0.5);
  int64_t o = v - B + L;
  o = o < 0 ? 0 : (o > 255 ? 255 : o);
  lut[(int64_t)c * 256 + v] = a.cflag[c] ? 0 : (uint8_t)o;
  if (v == 0 && chan_flags) chan_flags[c] = a.cflag[c];
}

__global__ __launch_bounds__(256) void k_emit_mask(RfiArgs a, uint8_t* mask) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < a.T) mask[t] = a.tflag[t] ? 0 : 1;
}

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

struct RfiLayout {
  int64_t rows = -1, rows_pitch = 0;
  int64_t m, b, r, cflag, z, tflag, keep8, keys, sel, nt, total;
};

RfiLayout rfi_layout(const sdd_plan* p, int64_t T) {
  RfiLayout L{};
  const int64_t C = p->nchan;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    const int64_t o = off;
    off += align256(bytes);
    return o;
  };
  if (p->layout == SDD_TIME_MAJOR) {
    L.rows_pitch = align256(T);
    L.rows = take(C * L.rows_pitch);
  }
  L.m = take(8 * C);
  L.b = take(8 * C);
  L.r = take(8 * C);
  L.cflag = take(4 * C);
  L.z = take(8 * T);
  L.tflag = take(4 * T);
  L.keep8 = take(T);
  L.keys = take(8 * std::max<int64_t>(C, T));
  L.sel = take(8 * 8);
  L.nt = take(8);
  L.total = off;
  return L;
}

// Rows of a pre-conditioned channel-major call sit past its workspace.
int64_t pre_rows_pitch(int64_t T) { return align256(T); }

}  // namespace
}  // namespace sdd

using namespace sdd;

extern "C" sdd_status sdd_rfi_workspace_size(const sdd_plan* p, int64_t nsamp_in, int64_t* bytes) {
  clear_error();
  if (!p || !bytes) SDD_FAIL(SDD_EINVAL, "null argument");
  if (nsamp_in < 1) SDD_FAIL(SDD_EINVAL, "nsamp_in must be >= 1");
  *bytes = rfi_layout(p, nsamp_in).total;
  return SDD_OK;
}

extern "C" sdd_status sdd_rfi_estimate(const sdd_plan* p, const uint8_t* d_in, int64_t nsamp_in,
                                       int64_t in_pitch, const sdd_rfi_desc* desc, uint8_t* d_lut,
                                       uint8_t* d_time_mask, int32_t* d_chan_flags, void* d_ws,
                                       int64_t ws_bytes, void* stream) {
  clear_error();
  if (!p || !d_in || !desc || !d_lut || !d_time_mask || !d_ws)
    SDD_FAIL(SDD_EINVAL, "null argument");
  if (nsamp_in < 1) SDD_FAIL(SDD_EINVAL, "nsamp_in must be >= 1");
  if (desc->median_window < 1 || desc->median_window > kMaxWindow || desc->median_window % 2 == 0)
    SDD_FAIL(SDD_EINVAL, "median_window must be odd, 1..%d", kMaxWindow);
  if (desc->rounds < 1 || desc->rounds > 16) SDD_FAIL(SDD_EINVAL, "rounds must be 1..16");
  if (!(desc->chan_sigma > 0.0) || !(desc->time_sigma > 0.0))
    SDD_FAIL(SDD_EINVAL, "thresholds must be positive");
  const int64_t minp = p->layout == SDD_TIME_MAJOR ? p->nchan : nsamp_in;
  if (in_pitch < minp) SDD_FAIL(SDD_EINVAL, "input pitch %lld < %lld", (long long)in_pitch,
                                (long long)minp);
  const RfiLayout L = rfi_layout(p, nsamp_in);
  if (ws_bytes < L.total)
    SDD_FAIL(SDD_ENOMEM, "workspace %lld bytes < %lld needed", (long long)ws_bytes,
             (long long)L.total);
  SDD_CHECK_WS_ALIGN(d_ws);
  DeviceGuard dg(p->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", p->device);
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w = (uint8_t*)d_ws;

  RfiArgs a{};
  a.C = p->nchan;
  a.T = nsamp_in;
  a.window = desc->median_window;
  a.k_chan = desc->chan_sigma;
  a.k_time = desc->time_sigma;
  if (p->layout == SDD_TIME_MAJOR) {
    SDD_HIP_TRY(launch_corner_turn(d_in, nsamp_in, in_pitch, p->nchan, w + L.rows, L.rows_pitch,
                                   s));
    a.rows = w + L.rows;
    a.pitch = L.rows_pitch;
  } else {
    a.rows = d_in;
    a.pitch = in_pitch;
  }
  a.m = (double*)(w + L.m);
  a.b = (double*)(w + L.b);
  a.r = (double*)(w + L.r);
  a.cflag = (int32_t*)(w + L.cflag);
  a.z = (int64_t*)(w + L.z);
  a.tflag = (int32_t*)(w + L.tflag);
  a.keep8 = w + L.keep8;
  a.keys = (uint64_t*)(w + L.keys);
  a.sel = (uint64_t*)(w + L.sel);
  a.nt = (int64_t*)(w + L.nt);

  const int64_t C = p->nchan, T = nsamp_in;
  const dim3 gC((unsigned)((C + 255) / 256)), gT((unsigned)((T + 255) / 256)), b256(256);
  const dim3 gZ((unsigned)((T + 1023) / 1024), (unsigned)((C + 63) / 64));
  const bool vec16 = (uintptr_t)a.rows % 16 == 0 && a.pitch % 16 == 0;
  const bool vec4 = (uintptr_t)a.rows % 4 == 0 && a.pitch % 4 == 0;
  // largest zero-DM sum C * 255 fixes how many key bytes the selections scan
  int ztop = 0;
  for (uint64_t zmax = (uint64_t)C * 255u; zmax >> (8 * (ztop + 1)); ++ztop) {
  }
  // no memset node: a caller may capture this sequence in a graph
  hipLaunchKernelGGL(k_clear_tflag, gT, b256, 0, s, a);
  for (int round = 0; round < desc->rounds; ++round) {
    hipLaunchKernelGGL(k_count_keep, dim3(1), dim3(1024), 0, s, a);
    if (vec16)
      hipLaunchKernelGGL(k_chan_mean<true>, dim3((unsigned)C), b256, 0, s, a);
    else
      hipLaunchKernelGGL(k_chan_mean<false>, dim3((unsigned)C), b256, 0, s, a);
    hipLaunchKernelGGL(k_bandpass, gC, b256, 0, s, a);
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, a.keys, C, (C - 1) / 2, 7, a.sel + 0);
    hipLaunchKernelGGL(k_absdev_f64, gC, b256, 0, s, a, (const double*)a.r, (int32_t)C,
                       (const uint64_t*)(a.sel + 0));
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, a.keys, C, (C - 1) / 2, 7, a.sel + 1);
    hipLaunchKernelGGL(k_cflag, gC, b256, 0, s, a);
    hipLaunchKernelGGL(k_clear_z, gT, b256, 0, s, a);
    if (vec4)
      hipLaunchKernelGGL(k_zero_dm<true>, gZ, b256, 0, s, a);
    else
      hipLaunchKernelGGL(k_zero_dm<false>, gZ, b256, 0, s, a);
    hipLaunchKernelGGL(k_z_keys, gT, b256, 0, s, a);
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, a.keys, T, (T - 1) / 2, ztop,
                       a.sel + 2);
    hipLaunchKernelGGL(k_absdev_i64, gT, b256, 0, s, a);
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, a.keys, T, (T - 1) / 2, ztop,
                       a.sel + 3);
    hipLaunchKernelGGL(k_tflag, gT, b256, 0, s, a);
  }
  hipLaunchKernelGGL(k_bp_keys, gC, b256, 0, s, a);
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, a.keys, C, (C - 1) / 2, 7, a.sel + 4);
  hipLaunchKernelGGL(k_emit_lut, dim3((unsigned)C), b256, 0, s, a, d_lut, d_chan_flags);
  hipLaunchKernelGGL(k_emit_mask, gT, b256, 0, s, a, d_time_mask);
  SDD_HIP_TRY(hipGetLastError());
  return SDD_OK;
}

extern "C" sdd_status sdd_pre_workspace_size(const sdd_plan* p, int64_t nsamp_in,
                                             int32_t lib_planes, int64_t* bytes) {
  clear_error();
  if (!p || !bytes) SDD_FAIL(SDD_EINVAL, "null argument");
  CallGeom cg;
  sdd_status st = plan_geometry(p, nsamp_in, &cg);
  if (st != SDD_OK) return st;
  int64_t need = lib_planes ? cg.ws.total_planes : cg.ws.total;
  if (p->layout == SDD_CHAN_MAJOR) need = align256(need) + p->nchan * pre_rows_pitch(nsamp_in);
  *bytes = need;
  return SDD_OK;
}

extern "C" sdd_status sdd_dedisperse_search_pre(
    const sdd_plan* p, const uint8_t* d_in, int64_t nsamp_in, int64_t in_pitch,
    const uint8_t* d_lut, const uint8_t* d_time_mask, uint32_t* const* d_planes,
    const int64_t* plane_pitch, sdd_dm_best* d_best, sdd_dm_stats* d_stats,
    sdd_candidate* d_cands, int32_t cap, int32_t* d_ncand, void* d_ws, int64_t ws_bytes,
    void* stream) {
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
  int64_t need = 0;
  if ((st = sdd_pre_workspace_size(p, nsamp_in, lib_planes ? 1 : 0, &need)) != SDD_OK) return st;
  if (ws_bytes < need || !d_ws)
    SDD_FAIL(SDD_ENOMEM, "workspace %lld bytes < %lld needed", (long long)ws_bytes,
             (long long)need);
  SDD_CHECK_WS_ALIGN(d_ws);
  uint32_t* own[SDD_MAX_RANGES];
  int64_t own_pitch[SDD_MAX_RANGES];
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
  Precond pre;
  pre.lut = d_lut;
  pre.tmask = d_time_mask;
  if (p->layout == SDD_CHAN_MAJOR) {
    const int64_t base = align256(lib_planes ? cg.ws.total_planes : cg.ws.total);
    pre.rows = (uint8_t*)d_ws + base;
    pre.rows_pitch = pre_rows_pitch(nsamp_in);
  }
  DeviceGuard dg(p->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", p->device);
  if ((st = plan_upload(p)) != SDD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = run_dedisperse(p, cg, d_in, nsamp_in, in_pitch, d_planes, plane_pitch, (uint8_t*)d_ws, s,
                      &pre);
  if (st != SDD_OK) return st;
  return run_search(p, cg, (const uint32_t* const*)d_planes, plane_pitch, d_best, d_stats,
                    d_cands, cap, d_ncand, (uint8_t*)d_ws, s);
}
