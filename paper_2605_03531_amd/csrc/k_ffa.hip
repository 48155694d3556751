// Fast Folding Algorithm (Section 3.5): each series is stacked as m rows of
// the base period p and turned into m folded profiles at the linearly spaced
// trial frequencies, then a circular boxcar filter finds the most significant
// pulse of every profile.
//
// Recursion (Staelin 1969, head/tail split for any height): a stack of
// len > 1 rows splits into h = len/2 head rows and t = len - h tail rows;
// profile s of the stack is head profile k_h plus tail profile k_t rolled by
// s - k_t bins, k_h = round(s(h-1)/(len-1)), k_t = round(s(t-1)/(len-1)).
// Every profile of a sub-stack is stored over the sub-stack's own rows, so a
// level of the recursion maps rows of one buffer to rows of another.
//
//   k_ffa_moments  exact uint64 S1/S2 of the m p folded samples per series
//   k_ffa_lds      the lowest levels: one workgroup per sub-stack that fits
//                  in LDS (ping-pong), from the input rows to its profiles
//   k_ffa_pass     one upper level through HBM: out[i] = A[a] + roll(A[b], sh)
//   k_ffa_boxcar   one wavefront per profile: circular uint64 prefix sums in
//                  LDS, each width's largest sum and first bin, FP64 S/N.
// Profiles are uint32 (the host checks m * max_value < 2^32), boxcar sums
// uint64: every sum is exact and every choice has a total order.
#include <algorithm>
#include <cmath>

#include "sdd_internal.h"

namespace sdd {
namespace {

constexpr int kThreads = 256;
constexpr int kLdsElems = 8192;  // u32 elements per LDS buffer of k_ffa_lds (two buffers)
constexpr int kLdsRows = 256;    // rows of a sub-stack of k_ffa_lds

struct FfaArgs {
  const uint32_t* in;  // series s at in + s * in_pitch
  int64_t in_pitch;
  int32_t nseries;
  int32_t p;
  int32_t m;
  int32_t nwidths;
  int32_t widths[SDD_MAX_WIDTHS];
  unsigned long long* moments;  // [nseries] {s1, s2}
  sdd_ffa_best* best;           // [nseries][m]
  sdd_dm_stats* stats;          // [nseries] or null
};

// Sub-stack of height len at recursion depth d (below a stack of height m)
// holding row i: lo, len. False if row i reaches a single row before depth d.
__device__ inline bool ffa_node(int32_t m, int32_t i, int d, int32_t* lo, int32_t* len) {
  int32_t l = 0, n = m;
  for (int k = 0; k < d; ++k) {
    if (n == 1) return false;
    const int32_t h = n >> 1;
    if (i < l + h) {
      n = h;
    } else {
      l += h;
      n -= h;
    }
  }
  *lo = l;
  *len = n;
  return true;
}

// Sources of row i at depth d: out[i][j] = src[a][j] + src[b][(j + sh) mod p]
// (b < 0: a copy of row a = i).
__device__ inline void ffa_sources(int32_t m, int32_t i, int d, int32_t p, int32_t* a,
                                   int32_t* b, int32_t* sh) {
  int32_t lo, len;
  if (!ffa_node(m, i, d, &lo, &len) || len == 1) {
    *a = i;
    *b = -1;
    *sh = 0;
    return;
  }
  const int32_t h = len >> 1, t = len - h;
  const int64_t s = i - lo, den = 2 * (int64_t)(len - 1);
  const int32_t kh = (int32_t)((2 * s * (h - 1) + (len - 1)) / den);
  const int32_t kt = (int32_t)((2 * s * (t - 1) + (len - 1)) / den);
  *a = lo + kh;
  *b = lo + h + kt;
  *sh = (int32_t)((s - kt) % p);
}

__global__ __launch_bounds__(256) void k_ffa_zero(unsigned long long* p, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) p[k] = 0ull;
}

__device__ inline unsigned long long wave_sum(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kThreads) void k_ffa_moments(FfaArgs a) {
  __shared__ unsigned long long red[2][kThreads / 64];
  const int32_t sr = blockIdx.y;
  const uint32_t* y = a.in + (int64_t)sr * a.in_pitch;
  const int64_t n = (int64_t)a.m * a.p;
  unsigned long long s1 = 0, s2 = 0;
  for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kThreads) {
    const unsigned long long v = y[j];
    s1 += v;
    s2 += v * v;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = s1;
    red[1][w] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t1 = 0, t2 = 0;
    for (int k = 0; k < kThreads / 64; ++k) {
      t1 += red[0][k];
      t2 += red[1][k];
    }
    atomicAdd(&a.moments[2 * sr], t1);
    atomicAdd(&a.moments[2 * sr + 1], t2);
  }
}

// Thread layout over rows of p bins: p >= 256 -> one row at a time, bins
// strided by 256; p < 256 -> R = 256 / p rows at a time, one bin each.
struct RowLane {
  int32_t r0, j0, rstep, jstep;
  bool on;
};
__device__ inline RowLane row_lane(int32_t p) {
  RowLane L;
  L.jstep = p >= kThreads ? kThreads : p;
  L.rstep = kThreads / L.jstep;
  L.r0 = (int32_t)threadIdx.x / L.jstep;
  L.j0 = (int32_t)threadIdx.x % L.jstep;
  L.on = L.r0 < L.rstep;
  return L;
}

// The lowest levels of one sub-stack (node `blockIdx.x` at depth d0, of at
// most kLdsRows and kLdsElems / p rows) from the input rows to its profiles, written to
// dst (series stride dst_pitch).
__global__ __launch_bounds__(kThreads) void k_ffa_lds(FfaArgs a, int d0, int32_t cap,
                                                      uint32_t* dst, int64_t dst_pitch) {
  extern __shared__ uint32_t sm[];  // 2 * cap, cap >= rows of the sub-stack * p
  __shared__ int32_t tab[3 * kLdsRows];
  const int32_t sr = blockIdx.y, p = a.p;
  // node index -> rows [lo, lo + len): bit d0-1-k of the index picks head or tail
  int32_t lo = 0, len = a.m;
  for (int k = 0; k < d0; ++k) {
    const int32_t h = len >> 1;
    if ((blockIdx.x >> (d0 - 1 - k)) & 1) {
      lo += h;
      len -= h;
    } else {
      len = h;
    }
  }
  const uint32_t* src = a.in + (int64_t)sr * a.in_pitch + (int64_t)lo * p;
  uint32_t* A = sm;
  uint32_t* B = sm + cap;
  const int32_t ne = len * p;
  // 8 loads in flight per thread before their LDS stores
  for (int32_t e0 = 0; e0 < ne; e0 += 8 * kThreads) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int32_t e = e0 + u * kThreads + (int32_t)threadIdx.x;
      v[u] = e < ne ? src[e] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int32_t e = e0 + u * kThreads + (int32_t)threadIdx.x;
      if (e < ne) A[e] = v[u];
    }
  }
  int depth = 0;  // levels of the sub-stack: ceil(log2 len)
  while ((1 << depth) < len) ++depth;
  const RowLane L = row_lane(p);
  for (int d = depth - 1; d >= 0; --d) {
    __syncthreads();  // A complete; previous readers of tab done
    for (int32_t r = threadIdx.x; r < len; r += kThreads)
      ffa_sources(len, r, d, p, &tab[3 * r], &tab[3 * r + 1], &tab[3 * r + 2]);
    __syncthreads();
    if (L.on)
      for (int32_t r = L.r0; r < len; r += L.rstep) {
        const int32_t ra = tab[3 * r], rb = tab[3 * r + 1], sh = tab[3 * r + 2];
        const uint32_t* pa = A + ra * p;
        uint32_t* po = B + r * p;
        if (rb < 0) {
          for (int32_t j = L.j0; j < p; j += L.jstep) po[j] = pa[j];
        } else {
          const uint32_t* pb = A + rb * p;
          for (int32_t j = L.j0; j < p; j += L.jstep) {
            int32_t k = j + sh;
            if (k >= p) k -= p;
            po[j] = pa[j] + pb[k];
          }
        }
      }
    uint32_t* t = A;
    A = B;
    B = t;
  }
  __syncthreads();
  uint32_t* out = dst + (int64_t)sr * dst_pitch + (int64_t)lo * p;
  for (int32_t e = threadIdx.x; e < ne; e += kThreads) out[e] = A[e];
}

// One upper level (depth d) through HBM: rows of src (series stride
// src_pitch) to rows of dst.
__global__ __launch_bounds__(kThreads) void k_ffa_pass(FfaArgs a, int d, const uint32_t* src,
                                                       int64_t src_pitch, uint32_t* dst,
                                                       int64_t dst_pitch) {
  const int32_t sr = blockIdx.y, p = a.p;
  const RowLane L = row_lane(p);
  if (!L.on) return;
  const int32_t i = (int32_t)blockIdx.x * L.rstep + L.r0;
  if (i >= a.m) return;
  int32_t ra, rb, sh;
  ffa_sources(a.m, i, d, p, &ra, &rb, &sh);
  const uint32_t* s = src + (int64_t)sr * src_pitch;
  const uint32_t* pa = s + (int64_t)ra * p;
  uint32_t* po = dst + (int64_t)sr * dst_pitch + (int64_t)i * p;
  if (rb < 0) {
    for (int32_t j = L.j0; j < p; j += L.jstep) po[j] = pa[j];
  } else {
    const uint32_t* pb = s + (int64_t)rb * p;
#pragma unroll 4
    for (int32_t j = L.j0; j < p; j += L.jstep) {
      int32_t k = j + sh;
      if (k >= p) k -= p;
      po[j] = pa[j] + pb[k];
    }
  }
}

// (B, j) order of one width: the larger sum, then the smaller bin.
__device__ inline bool bj_better(unsigned long long b, int32_t j, unsigned long long b2,
                                 int32_t j2) {
  return b > b2 || (b == b2 && j < j2);
}

// mu = S1/n, sigma = sqrt(n S2 - S1^2)/n with the numerator exact (128-bit).
__device__ inline void fold_mean_sigma(uint64_t n, uint64_t s1, uint64_t s2, double* mu,
                                       double* sigma) {
  const uint64_t p_lo = n * s2, p_hi = __umul64hi(n, s2);
  const uint64_t q_lo = s1 * s1, q_hi = __umul64hi(s1, s1);
  const uint64_t d_lo = p_lo - q_lo;
  const uint64_t d_hi = p_hi - q_hi - (p_lo < q_lo ? 1ull : 0ull);
  *mu = (double)s1 / (double)n;
  *sigma = 0.0;
  if (d_hi != 0 || d_lo != 0)
    *sigma = sqrt((double)d_hi * 18446744073709551616.0 + (double)d_lo) / (double)n;
}

// Best (S/N, bin, width) of folded profiles: one wavefront per profile
// (profile 4 * blockIdx.x + wave of series blockIdx.y). Lane l sums its
// chunk of ceil(p / 64) consecutive bins; a wave scan of the chunk sums gives
// P[k] = sum of bins < k in LDS (P[p] the total), and the circular boxcar
// from bin j is P[j + w] - P[j], or P[p] - P[j] + P[j + w - p] past the end.
// Per width the largest sum and its first bin (wave reduction), then FP64
// S/N, compared in the F6 order as the widths go.
__global__ __launch_bounds__(kThreads) void k_ffa_boxcar(FfaArgs a, const uint32_t* prof,
                                                         int64_t prof_pitch) {
  extern __shared__ unsigned long long P_all[];  // 4 x (p + 1)
  const int32_t p = a.p, sr = blockIdx.y;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int32_t s = (int32_t)blockIdx.x * (kThreads / 64) + wid;
  if (s >= a.m) return;  // whole wavefront: no workgroup barrier below
  unsigned long long* P = P_all + (int64_t)wid * (p + 1);
  const uint32_t* row = prof + (int64_t)sr * prof_pitch + (int64_t)s * p;
  const int32_t c = (p + 63) / 64;
  const int32_t k0 = min(lane * c, p), k1 = min(k0 + c, p);
  unsigned long long part = 0;
#pragma unroll 4
  for (int32_t k = k0; k < k1; ++k) part += row[k];
  unsigned long long inc = part;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  unsigned long long off = inc - part;
  for (int32_t k = k0; k < k1; ++k) {
    P[k] = off;
    off += row[k];
  }
  const unsigned long long total = __shfl(inc, 63, 64);
  if (lane == 0) P[p] = total;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint64_t n = (uint64_t)a.m * (uint64_t)p;
  double mu, sigma;
  fold_mean_sigma(n, a.moments[2 * sr], a.moments[2 * sr + 1], &mu, &sigma);
  double bs = 0.0;
  int32_t bj = 0, bw = a.widths[0];
  if (sigma > 0.0) {
    bs = -INFINITY;
    for (int q = 0; q < a.nwidths; ++q) {
      const int32_t w = a.widths[q];
      unsigned long long bb = 0ull;
      int32_t bjj = 0x7fffffff;
      for (int32_t j = lane; j < p; j += 64) {
        const int32_t e = j + w;
        const unsigned long long b = e <= p ? P[e] - P[j] : total - P[j] + P[e - p];
        if (bj_better(b, j, bb, bjj)) {
          bb = b;
          bjj = j;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long b2 = __shfl_xor(bb, o, 64);
        const int32_t j2 = __shfl_xor(bjj, o, 64);
        if (bj_better(b2, j2, bb, bjj)) {
          bb = b2;
          bjj = j2;
        }
      }
      const double sn =
          ((double)bb - (double)w * (double)a.m * mu) / (sigma * sqrt((double)a.m * (double)w));
      if (sn > bs || (sn == bs && bjj < bj)) {  // widths ascend: a tie keeps the smaller
        bs = sn;
        bj = bjj;
        bw = w;
      }
    }
  }
  if (lane == 0) {
    sdd_ffa_best o;
    o.snr = (float)bs;
    o.bin = bj;
    o.width = bw;
    o.pad = 0;
    a.best[(int64_t)sr * a.m + s] = o;
    if (s == 0 && a.stats) {
      sdd_dm_stats st;
      st.n = (int64_t)n;
      st.s1 = a.moments[2 * sr];
      st.s2 = a.moments[2 * sr + 1];
      st.mean = mu;
      st.std = sigma;
      a.stats[sr] = st;
    }
  }
}

int floor_log2(int64_t v) {
  int d = 0;
  while (((int64_t)2 << d) <= v) ++d;
  return d;
}

int64_t round_up256(int64_t v) { return (v + 255) & ~(int64_t)255; }

struct FfaLayout {
  int64_t moments = 0, buf0 = 0, buf1 = 0, total = 0;
};

FfaLayout ffa_layout(int32_t nseries, int64_t m, int32_t p) {
  FfaLayout L;
  L.moments = 0;
  int64_t off = round_up256((int64_t)nseries * 16);
  const int64_t stack = round_up256((int64_t)nseries * m * p * 4);
  L.buf0 = off;
  L.buf1 = off + stack;
  L.total = off + 2 * stack;
  return L;
}

}  // namespace
}  // namespace sdd

using namespace sdd;

extern "C" sdd_status sdd_ffa_workspace_size(int32_t nseries, int64_t nsamp, int32_t period,
                                             int64_t* bytes) {
  clear_error();
  if (!bytes || nseries < 1 || period < 2 || nsamp < period)
    SDD_FAIL(SDD_EINVAL, "need nseries >= 1, period >= 2, nsamp >= period and bytes");
  *bytes = ffa_layout(nseries, nsamp / period, period).total;
  return SDD_OK;
}

extern "C" sdd_status sdd_ffa_search(int32_t device, const uint32_t* d_series, int64_t pitch,
                                     int32_t nseries, int64_t nsamp, int32_t period,
                                     uint32_t max_value, const int32_t* widths, int32_t nwidths,
                                     uint32_t* d_profiles, sdd_ffa_best* d_best,
                                     sdd_dm_stats* d_stats, void* d_ws, int64_t ws_bytes,
                                     void* stream) {
  clear_error();
  if (!d_series || !d_best || !d_ws || !widths)
    SDD_FAIL(SDD_EINVAL, "null series, best, workspace or widths");
  if (nseries < 1 || period < 2 || period > SDD_FFA_MAX_PERIOD || nsamp < period ||
      pitch < nsamp)
    SDD_FAIL(SDD_EINVAL, "need nseries >= 1, 2 <= period <= %d, nsamp >= period, pitch >= nsamp",
             SDD_FFA_MAX_PERIOD);
  if (nwidths < 1 || nwidths > SDD_MAX_WIDTHS)
    SDD_FAIL(SDD_EINVAL, "nwidths must be in [1, %d]", SDD_MAX_WIDTHS);
  for (int32_t k = 0; k < nwidths; ++k)
    if (widths[k] < 1 || widths[k] >= period || (k > 0 && widths[k] <= widths[k - 1]))
      SDD_FAIL(SDD_EINVAL, "widths must increase strictly within 1..period-1");
  const int64_t m = nsamp / period;
  if (m >= (int64_t)1 << 24 || nseries > 65535)
    SDD_FAIL(SDD_EINVAL, "at most 2^24 - 1 rows and 65535 series per call");
  if ((long double)m * max_value >= 4294967296.0L)
    SDD_FAIL(SDD_ERANGE, "m * max_value = %lld * %u could overflow a 32-bit profile bin",
             (long long)m, max_value);
  if ((long double)m * period * (long double)max_value * max_value >= 18446744073709551615.0L)
    SDD_FAIL(SDD_ERANGE, "the 64-bit sum of squares could overflow");
  const FfaLayout lay = ffa_layout(nseries, m, period);
  if (ws_bytes < lay.total)
    SDD_FAIL(SDD_ENOMEM, "FFA workspace needs %lld bytes", (long long)lay.total);
  DeviceGuard dg(device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", device);
  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)d_ws;

  FfaArgs a{};
  a.in = d_series;
  a.in_pitch = pitch;
  a.nseries = nseries;
  a.p = period;
  a.m = (int32_t)m;
  a.nwidths = nwidths;
  for (int32_t k = 0; k < nwidths; ++k) a.widths[k] = widths[k];
  a.moments = reinterpret_cast<unsigned long long*>(ws + lay.moments);
  a.best = d_best;
  a.stats = d_stats;

  StageTimer tm(SDD_STAGE_FFA, s);
  hipLaunchKernelGGL(k_ffa_zero, dim3((unsigned)((2 * (int64_t)nseries + 255) / 256)), dim3(256),
                     0, s, a.moments, 2 * (int64_t)nseries);
  const int64_t nfold = m * period;
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, nfold / 8192));
  hipLaunchKernelGGL(k_ffa_moments, dim3(gx, (unsigned)nseries), dim3(kThreads), 0, s, a);

  // lowest levels in LDS: the shallowest depth whose sub-stacks fit (every
  // row still belongs to a sub-stack there: depth <= floor(log2 m))
  int d0 = 0;
  auto height = [&](int d) { return (m + ((int64_t)1 << d) - 1) >> d; };
  while (d0 < floor_log2(m) && (height(d0) * period > kLdsElems || height(d0) > kLdsRows)) ++d0;
  const int64_t stack = m * period;
  uint32_t* bufs[2] = {reinterpret_cast<uint32_t*>(ws + lay.buf0),
                       reinterpret_cast<uint32_t*>(ws + lay.buf1)};
  // destinations: the final level writes d_profiles when given; the others
  // alternate between the two workspace stacks
  auto dst_of = [&](int k, int nlev) -> uint32_t* {
    if (k == nlev - 1 && d_profiles) return d_profiles;
    return bufs[k & 1];
  };
  const int nlev = 1 + d0;  // the LDS kernel, then the passes at depths d0-1 .. 0
  uint32_t* cur = dst_of(0, nlev);
  const int32_t cap = (int32_t)(height(d0) * period);
  const size_t lds_a = 2 * (size_t)cap * sizeof(uint32_t);
  const size_t lds_b = (size_t)(kThreads / 64) * (period + 1) * sizeof(unsigned long long);
  // at most 64 KiB and 4 x 4097 x 8 bytes: within gfx950's 160 KiB per workgroup
  SDD_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ffa_lds),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 65536));
  SDD_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ffa_boxcar),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_b));
  hipLaunchKernelGGL(k_ffa_lds, dim3(1u << d0, (unsigned)nseries), dim3(kThreads), lds_a, s, a,
                     d0, cap, cur, stack);
  const int32_t rstep = period >= kThreads ? 1 : kThreads / period;
  for (int k = 1; k < nlev; ++k) {
    uint32_t* nxt = dst_of(k, nlev);
    hipLaunchKernelGGL(k_ffa_pass, dim3((unsigned)((m + rstep - 1) / rstep), (unsigned)nseries),
                       dim3(kThreads), 0, s, a, d0 - k, cur, stack, nxt, stack);
    cur = nxt;
  }
  hipLaunchKernelGGL(k_ffa_boxcar, dim3((unsigned)((m + 3) / 4), (unsigned)nseries),
                     dim3(kThreads), lds_b, s, a, cur, stack);
  SDD_HIP_TRY(hipGetLastError());
  return SDD_OK;
}
