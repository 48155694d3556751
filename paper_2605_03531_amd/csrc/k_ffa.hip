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
//   k_ffa_boxcar   one segment of 16 or 64 lanes per profile: circular prefix
//                  sums in LDS, each width's largest sum and first bin, FP64 S/N.
// Profiles are uint32 (the host checks m * max_value < 2^32), boxcar sums
// uint64: every sum is exact and every choice has a total order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "sdd_internal.h"

namespace sdd {
namespace {

constexpr int kThreads = 256;
constexpr int kLdsElems = 8192;  // u32 elements per LDS buffer of k_ffa_lds (two buffers)
constexpr int kLdsRows = 256;    // rows of a sub-stack of k_ffa_lds
constexpr int kLdsThreads = 1024; // workgroup of k_ffa_lds

struct FfaArgs {
  const uint32_t* in;  // series s at in + s * in_pitch
  int64_t in_pitch;
  int32_t nseries;
  int32_t p;
  int32_t m;
  int32_t nwidths;
  int32_t widths[SDD_MAX_WIDTHS];
  unsigned long long* moments;  // [nseries] {s1, s2}
  const int4* tab;              // [depth][m] sources of every row at the HBM-pass depths
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

// Thread layout over rows of p bins for a workgroup of T threads: p >= T ->
// one row at a time, bins strided by T; p < T -> R = T / p rows at a time,
// one bin each.
struct RowLane {
  int32_t r0, j0, rstep, jstep;
  bool on;
};
template <int T = kThreads>
__device__ inline RowLane row_lane(int32_t p) {
  RowLane L;
  L.jstep = p >= T ? T : p;
  L.rstep = T / L.jstep;
  L.r0 = (int32_t)threadIdx.x / L.jstep;
  L.j0 = (int32_t)threadIdx.x % L.jstep;
  L.on = L.r0 < L.rstep;
  return L;
}

// The lowest levels of one sub-stack (node `blockIdx.x` at depth d0, of at
// most kLdsRows and kLdsElems / p rows) from the input rows to its profiles,
// written to dst (series stride dst_pitch).
__global__ __launch_bounds__(kLdsThreads) void k_ffa_lds(FfaArgs a, int d0, int32_t cap,
                                                         uint32_t* dst, int64_t dst_pitch) {
  extern __shared__ uint32_t sm[];  // 2 * cap, cap >= rows of the sub-stack * p
  // per (level, row): a | b << 8 | copy << 16 | roll << 17 (rows < 256, roll < 4096)
  __shared__ uint32_t tab[8 * kLdsRows];
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
  for (int32_t e0 = 0; e0 < ne; e0 += 8 * kLdsThreads) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int32_t e = e0 + u * kLdsThreads + (int32_t)threadIdx.x;
      v[u] = e < ne ? src[e] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int32_t e = e0 + u * kLdsThreads + (int32_t)threadIdx.x;
      if (e < ne) A[e] = v[u];
    }
  }
  int depth = 0;  // levels of the sub-stack: ceil(log2 len) <= 8
  while ((1 << depth) < len) ++depth;
  for (int32_t k = threadIdx.x; k < depth * len; k += kLdsThreads) {
    const int d = k / len;
    const int32_t r = k - d * len;
    int32_t ra, rb, sh;
    ffa_sources(len, r, d, p, &ra, &rb, &sh);
    tab[k] = (uint32_t)ra | (rb < 0 ? 1u << 16 : (uint32_t)rb << 8) | ((uint32_t)sh << 17);
  }
  const RowLane L = row_lane<kLdsThreads>(p);
  for (int d = depth - 1; d >= 0; --d) {
    __syncthreads();  // A (and at the first level the table) complete
    if (L.on)
      for (int32_t r = L.r0; r < len; r += L.rstep) {
        const uint32_t t = tab[d * len + r];
        const int32_t ra = (int32_t)(t & 255u), sh = (int32_t)(t >> 17);
        const int32_t rb = (t >> 16) & 1u ? -1 : (int32_t)((t >> 8) & 255u);
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
  for (int32_t e = threadIdx.x; e < ne; e += kLdsThreads) out[e] = A[e];
}

// Sources of every row for the HBM passes, once per call: entry (d, i) of
// [d0][m] pairs of int4. A single level at depth d: {a, b, roll}; two levels
// at depths d and d + 1 (rows at depth d + 2 in, depth d out):
// out[i][j] = X[a1][j] + X[a2][j + ra] + X[b1][j + rb] + X[b2][j + rbb]
// (indices mod p), {a1, a2, b1, b2}, {ra, rb, rbb, 0}. Depths below d0 have
// no copies (every sub-stack there has two or more rows).
__global__ __launch_bounds__(256) void k_ffa_table(int32_t m, int32_t p, int d0, int4* tab) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= (int64_t)d0 * m) return;
  const int d = (int)(k / m);
  const int32_t i = (int32_t)(k - (int64_t)d * m);
  int32_t a, b, r;
  ffa_sources(m, i, d, p, &a, &b, &r);
  int4 t0 = make_int4(a, b, r, 0), t1 = make_int4(0, 0, 0, 0);
  if (d + 1 < d0) {
    int32_t a1, a2, ra, b1, b2, rb;
    ffa_sources(m, a, d + 1, p, &a1, &a2, &ra);
    ffa_sources(m, b, d + 1, p, &b1, &b2, &rb);
    t0 = make_int4(a1, a2, b1, b2);
    t1 = make_int4(ra, r, (int32_t)(((int64_t)r + rb) % p), 0);
  }
  tab[2 * k] = t0;
  tab[2 * k + 1] = t1;
}

// One upper level (depth d) through HBM: rows of src (series stride
// src_pitch) to rows of dst; workgroup blockIdx.x of gridDim.x walks every
// gridDim.x-th group of rows of series blockIdx.y.
// TWO: levels d and d + 1 at once (four rows in, one out).
template <bool TWO>
__global__ __launch_bounds__(kThreads) void k_ffa_pass(FfaArgs a, int d, const uint32_t* src,
                                                       int64_t src_pitch, uint32_t* dst,
                                                       int64_t dst_pitch) {
  const int32_t sr = blockIdx.y, p = a.p;
  const RowLane L = row_lane(p);
  if (!L.on) return;
  const uint32_t* s = src + (int64_t)sr * src_pitch;
  for (int32_t i = (int32_t)blockIdx.x * L.rstep + L.r0; i < a.m;
       i += (int32_t)gridDim.x * L.rstep) {
    const int4 t0 = a.tab[2 * ((int64_t)d * a.m + i)];
    uint32_t* po = dst + (int64_t)sr * dst_pitch + (int64_t)i * p;
    if constexpr (TWO) {
      const int4 t1 = a.tab[2 * ((int64_t)d * a.m + i) + 1];
      const uint32_t* p0 = s + (int64_t)t0.x * p;
      const uint32_t* p1 = s + (int64_t)t0.y * p;
      const uint32_t* p2 = s + (int64_t)t0.z * p;
      const uint32_t* p3 = s + (int64_t)t0.w * p;
#pragma unroll 4
      for (int32_t j = L.j0; j < p; j += L.jstep) {
        int32_t k1 = j + t1.x, k2 = j + t1.y, k3 = j + t1.z;
        if (k1 >= p) k1 -= p;
        if (k2 >= p) k2 -= p;
        if (k3 >= p) k3 -= p;
        po[j] = p0[j] + p1[k1] + p2[k2] + p3[k3];
      }
    } else {
      const int32_t ra = t0.x, rb = t0.y, sh = t0.z;
      const uint32_t* pa = s + (int64_t)ra * p;
      const uint32_t* pb = s + (int64_t)rb * p;
#pragma unroll 4
      for (int32_t j = L.j0; j < p; j += L.jstep) {
        int32_t k = j + sh;
        if (k >= p) k -= p;
        po[j] = pa[j] + pb[k];
      }
    }
  }
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

// (S/N, bin, width) order of the search: the larger S/N, then the smaller
// bin, then the smaller width.
__device__ inline bool snr_better(double s, int32_t j, int32_t w, double s2, int32_t j2,
                                  int32_t w2) {
  return s > s2 || (s == s2 && (j < j2 || (j == j2 && w < w2)));
}

// Best (S/N, bin, width) of folded profiles: one segment of W lanes per
// profile (64 / W profiles per wavefront, so short profiles share a
// wavefront's fixed costs); segment g of the workgroup takes profiles
// g + G * gridDim.x * k of series blockIdx.y (G segments per workgroup).
// Lane l of a segment sums its chunk of ceil(p / W) consecutive bins; a
// segment scan of the chunk sums gives P[k] = sum of bins < k in LDS (P[p]
// the total), and the circular boxcar from bin j is P[j + w] - P[j], or
// P[p] - P[j] + P[j + w - p] past the end. Each lane keeps, per width, the
// largest sum over its bins (first bin on ties: its bins ascend), turns it
// into the FP64 S/N (B - w m mu) / (sigma sqrt(m w)) and keeps its best in
// the search's order; one segment reduction in the same order ends the
// profile. Shuffles never leave a segment, whose lanes share one profile.
template <int W>
__global__ __launch_bounds__(kThreads) void k_ffa_boxcar(FfaArgs a, const uint32_t* prof,
                                                         int64_t prof_pitch) {
  // G x (p + 1) u64: per segment a u64 prefix, or a u32 prefix of p + w_max
  extern __shared__ unsigned long long P_all[];
  __shared__ double wnum[SDD_MAX_WIDTHS], wden[SDD_MAX_WIDTHS];
  constexpr int G = kThreads / W;  // segments per workgroup
  const int32_t p = a.p, sr = blockIdx.y;
  const int lane = threadIdx.x % W, seg = threadIdx.x / W;
  unsigned long long* P = P_all + (int64_t)seg * (p + 1);
  const uint64_t n = (uint64_t)a.m * (uint64_t)p;
  double mu, sigma;
  fold_mean_sigma(n, a.moments[2 * sr], a.moments[2 * sr + 1], &mu, &sigma);
  if (threadIdx.x < (unsigned)a.nwidths) {
    const double w = (double)a.widths[threadIdx.x];
    wnum[threadIdx.x] = w * (double)a.m * mu;
    wden[threadIdx.x] = sigma * sqrt((double)a.m * w);
  }
  __syncthreads();
  // each segment loops on its own: no workgroup barrier below
  for (int32_t s = (int32_t)blockIdx.x * G + seg; s < a.m; s += (int32_t)gridDim.x * G) {
    const uint32_t* row = prof + (int64_t)sr * prof_pitch + (int64_t)s * p;
    // the previous profile's readers of P are done
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t c = (p + W - 1) / W;
    const int32_t k0 = min(lane * c, p), k1 = min(k0 + c, p);
    unsigned long long part = 0;
    uint32_t lmin = 0xffffffffu;
#pragma unroll 4
    for (int32_t k = k0; k < k1; ++k) {
      const uint32_t v = row[k];
      part += v;
      lmin = min(lmin, v);
    }
    unsigned long long inc = part;
    for (int o = 1; o < W; o <<= 1) {
      const unsigned long long t = __shfl_up(inc, o, W);
      if (lane >= o) inc += t;
    }
    for (int o = W / 2; o > 0; o >>= 1) lmin = min(lmin, (uint32_t)__shfl_xor((int)lmin, o, W));
    const uint32_t base = lmin;  // the profile's smallest bin
    const unsigned long long total = __shfl(inc, W - 1, W);
    // bins minus the smallest one: when their total fits 32 bits (the usual
    // case) the prefix of the offset bins is exact in uint32 and every boxcar
    // of them too; B = B' + w * base
    const bool narrow = total - (unsigned long long)p * base < (1ull << 32);
    double bs = 0.0;
    int32_t bj = 0, bw = a.widths[0];
    if (narrow) {
      uint32_t* Q = reinterpret_cast<uint32_t*>(P);  // p + w_max entries
      uint32_t off = (uint32_t)(inc - part) - (uint32_t)k0 * base;
      for (int32_t k = k0; k < k1; ++k) {
        Q[k] = off;
        off += row[k] - base;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // circular extension: Q[p + k] = Q[p] + Q[k]
      const uint32_t qtot = (uint32_t)(total - (unsigned long long)p * base);
      const int32_t wmax = a.widths[a.nwidths - 1];
      for (int32_t k = lane; k < wmax; k += W) Q[p + k] = qtot + Q[k];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (sigma > 0.0) {
        bs = -INFINITY;
        bj = 0x7fffffff;
        for (int q0 = 0; q0 < a.nwidths; q0 += 8) {
          uint32_t bb[8];
          int32_t bjj[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            bb[u] = 0u;
            bjj[u] = -1;
          }
          for (int32_t j = lane; j < p; j += W) {
            const uint32_t qj = Q[j];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              if (q0 + u < a.nwidths) {
                const uint32_t b = Q[j + a.widths[q0 + u]] - qj;
                if (bjj[u] < 0 || b > bb[u]) {
                  bb[u] = b;
                  bjj[u] = j;
                }
              }
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (q0 + u < a.nwidths && bjj[u] >= 0) {
              const int32_t w = a.widths[q0 + u];
              const unsigned long long B = (unsigned long long)bb[u] + (unsigned long long)w * base;
              const double sn = ((double)B - wnum[q0 + u]) / wden[q0 + u];
              if (snr_better(sn, bjj[u], w, bs, bj, bw)) {
                bs = sn;
                bj = bjj[u];
                bw = w;
              }
            }
          }
        }
      }
    } else {
      unsigned long long off = inc - part;
      for (int32_t k = k0; k < k1; ++k) {
        P[k] = off;
        off += row[k];
      }
      if (lane == 0) P[p] = total;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (sigma > 0.0) {
        bs = -INFINITY;
        bj = 0x7fffffff;
        for (int q = 0; q < a.nwidths; ++q) {
          const int32_t w = a.widths[q];
          unsigned long long bb = 0ull;
          int32_t bjj = -1;
          for (int32_t j = lane; j < p; j += W) {
            const int32_t e = j + w;
            const unsigned long long b = e <= p ? P[e] - P[j] : total - P[j] + P[e - p];
            if (bjj < 0 || b > bb) {
              bb = b;
              bjj = j;
            }
          }
          if (bjj >= 0) {
            const double sn = ((double)bb - wnum[q]) / wden[q];
            if (snr_better(sn, bjj, w, bs, bj, bw)) {
              bs = sn;
              bj = bjj;
              bw = w;
            }
          }
        }
      }
    }
    if (sigma > 0.0) {
      for (int o = W / 2; o > 0; o >>= 1) {
        const double s2 = __shfl_xor(bs, o, W);
        const int32_t j2 = __shfl_xor(bj, o, W);
        const int32_t w2 = __shfl_xor(bw, o, W);
        if (snr_better(s2, j2, w2, bs, bj, bw)) {
          bs = s2;
          bj = j2;
          bw = w2;
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
}

int floor_log2(int64_t v) {
  int d = 0;
  while (((int64_t)2 << d) <= v) ++d;
  return d;
}

int64_t round_up256(int64_t v) { return (v + 255) & ~(int64_t)255; }

struct FfaLayout {
  int64_t moments = 0, tab = 0, buf0 = 0, buf1 = 0, total = 0;
};

// Depth of the sub-stacks that k_ffa_lds folds: the shallowest whose
// sub-stacks hold at most kLdsRows rows and kLdsElems bins (every row still
// belongs to a sub-stack there: depth <= floor(log2 m)). The levels above it
// are the HBM passes.
int lds_depth(int64_t m, int32_t p) {
  auto height = [&](int d) { return (m + ((int64_t)1 << d) - 1) >> d; };
  int d0 = 0;
  while (d0 < floor_log2(m) && (height(d0) * p > kLdsElems || height(d0) > kLdsRows)) ++d0;
  return d0;
}

// moments [nseries] x 16 B, source tables [d0][m] x 32 B, two stacks
FfaLayout ffa_layout(int32_t nseries, int64_t m, int32_t p) {
  FfaLayout L;
  L.moments = 0;
  L.tab = round_up256((int64_t)nseries * 16);
  int64_t off = L.tab + round_up256((int64_t)lds_depth(m, p) * m * 32);
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
  SDD_CHECK_WS_ALIGN(d_ws);
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

  const int d0 = lds_depth(m, period);
  auto height = [&](int d) { return (m + ((int64_t)1 << d) - 1) >> d; };
  const int64_t stack = m * period;
  a.tab = reinterpret_cast<const int4*>(ws + lay.tab);
  if (d0 > 0)
    hipLaunchKernelGGL(k_ffa_table, dim3((unsigned)(((int64_t)d0 * m + 255) / 256)), dim3(256), 0,
                       s, (int32_t)m, period, d0, reinterpret_cast<int4*>(ws + lay.tab));
  uint32_t* bufs[2] = {reinterpret_cast<uint32_t*>(ws + lay.buf0),
                       reinterpret_cast<uint32_t*>(ws + lay.buf1)};
  // destinations: the final level writes d_profiles when given; the others
  // alternate between the two workspace stacks
  auto dst_of = [&](int k, int nlev) -> uint32_t* {
    if (k == nlev - 1 && d_profiles) return d_profiles;
    return bufs[k & 1];
  };
  // the HBM levels d0-1 .. 0: one single-level pass first when d0 is odd,
  // then passes of two levels each (the tables hold the matching entries)
  struct Step {
    int depth;  // depth of the rows the pass writes
    bool two;
  };
  std::vector<Step> steps;
  for (int dc = d0; dc > 0;) {
    const bool two = !(dc == d0 && (d0 & 1));
    steps.push_back({dc - (two ? 2 : 1), two});
    dc -= two ? 2 : 1;
  }
  const int nlev = 1 + (int)steps.size();  // the LDS kernel, then the passes
  uint32_t* cur = dst_of(0, nlev);
  const int32_t cap = (int32_t)(height(d0) * period);
  const size_t lds_a = 2 * (size_t)cap * sizeof(uint32_t);
  // segment of W lanes per profile: profiles of up to 256 bins share a
  // wavefront four at a time (measured: 2.8x faster at 128 bins; 32-lane
  // segments were slower at 1024 bins than whole wavefronts)
  const int wseg = period <= 256 ? 16 : 64;
  const size_t lds_b = (size_t)(kThreads / wseg) * (period + 1) * sizeof(unsigned long long);
  // at most 64 KiB and 4 x 4097 x 8 bytes: within gfx950's 160 KiB per workgroup
  SDD_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ffa_lds),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 65536));
  const void* box = wseg == 16 ? reinterpret_cast<const void*>(&k_ffa_boxcar<16>)
                               : reinterpret_cast<const void*>(&k_ffa_boxcar<64>);
  SDD_HIP_TRY(hipFuncSetAttribute(box, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_b));
  hipLaunchKernelGGL(k_ffa_lds, dim3(1u << d0, (unsigned)nseries), dim3(kLdsThreads), lds_a, s,
                     a, d0, cap, cur, stack);
  // about 32K workgroups per pass, each with at least 16 elements per thread
  const int32_t rstep = period >= kThreads ? 1 : kThreads / period;
  const int64_t groups = (m + rstep - 1) / rstep;
  const int64_t per_grp = (int64_t)rstep * period;  // elements of one row group
  const int64_t gx_pass = std::max<int64_t>(
      1, std::min<int64_t>({groups, (32768 + nseries - 1) / nseries,
                            (groups * per_grp) / (16 * kThreads) + 1}));
  for (int k = 1; k < nlev; ++k) {
    uint32_t* nxt = dst_of(k, nlev);
    const Step& st = steps[k - 1];
    if (st.two)
      hipLaunchKernelGGL(k_ffa_pass<true>, dim3((unsigned)gx_pass, (unsigned)nseries),
                         dim3(kThreads), 0, s, a, st.depth, cur, stack, nxt, stack);
    else
      hipLaunchKernelGGL(k_ffa_pass<false>, dim3((unsigned)gx_pass, (unsigned)nseries),
                         dim3(kThreads), 0, s, a, st.depth, cur, stack, nxt, stack);
    cur = nxt;
  }
  const int64_t per_wg = kThreads / wseg;  // profiles in flight per workgroup
  const int64_t gx_box = std::max<int64_t>(
      1, std::min<int64_t>((m + per_wg - 1) / per_wg, (16384 + nseries - 1) / nseries));
  const dim3 gbox((unsigned)gx_box, (unsigned)nseries);
  if (wseg == 16)
    hipLaunchKernelGGL(k_ffa_boxcar<16>, gbox, dim3(kThreads), lds_b, s, a, cur, stack);
  else
    hipLaunchKernelGGL(k_ffa_boxcar<64>, gbox, dim3(kThreads), lds_b, s, a, cur, stack);
  SDD_HIP_TRY(hipGetLastError());
  return SDD_OK;
}
