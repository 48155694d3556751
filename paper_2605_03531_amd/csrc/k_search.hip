// Single-pulse search by time-domain boxcar filtering (Section 2.1) over the
// dedispersed DM-time planes:
//   k_seg      one wavefront per 1024 owned starts of one trial (cells of a
//              multiple of 1024 starts): samples in registers, wrap-around
//              uint32 prefix sums by a wave scan into LDS, B_w[j] = P[j+w] -
//              P[j] exactly; per width the maximum and first argmax; exact
//              uint64 S1/S2 of the owned samples, accumulated per trial with
//              integer atomics.
//   k_cells    the same per (trial, cell) for any cell size, one workgroup
//              per cell (used when k_seg's layout conditions do not hold).
//   k_rows     per trial: FP64 mean/sigma from the exact moments, S/N of each
//              cell's per-width maxima, the cell's best, the trial's best and
//              its candidate count (S/N > threshold).
//   k_scan     exclusive scan of the per-trial counts (one workgroup).
//   k_compact  per trial: writes its candidates in sample order at its offset.
// With de-reddening (Section 3.3) k_dered_base first finds each trial's
// block baselines (running median in block strides), and every kernel that
// reads the plane searches clip(y - base + M/2, 0, M) instead of y.
// Every step is deterministic: integer sums are order-free and every
// selection has a total tie order.
#include <algorithm>
#include <cmath>

#include "sdd_internal.h"

namespace sdd {
namespace {

constexpr int kThreads = 256;
constexpr int kSub = 1024;  // owned starts per LDS sub-segment

// Per (cell, width) result: (max B << 32) | ~(first argmax - cell start),
// so the larger key is the larger sum, then the earlier start.
using CellKey = unsigned long long;
struct CellBest {
  double snr;
  int32_t j;
  uint32_t wf;  // width | (candidate << 31)
};
struct Moments {
  unsigned long long s1, s2;
};

__device__ inline int find_range(const SearchArgs& a, int32_t g) {
  int r = 0;
  for (int k = 1; k < a.nranges; ++k)
    if (g >= a.r[k].dm_offset) r = k;
  return r;
}

__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long t = __shfl_xor(v, o, 64);
    v = t > v ? t : v;
  }
  return v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive scan over the workgroup (kThreads threads); tmp holds one entry
// per wavefront. Contains two barriers.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T* tmp, T* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    T t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) tmp[wid] = inc;
  __syncthreads();
  T off = 0, tot = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    T t = tmp[w];
    if (w < wid) off += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// ---- de-reddening (running-median subtraction, Section 3.3) ---------------
// The searched sample: y - base + M/2 clipped to [0, M], M the plane's full
// scale, so every bound of the plain plane still holds.
__device__ inline uint32_t dered(uint32_t y, uint32_t base, int32_t M) {
  const int32_t t = (int32_t)y - (int32_t)base + (M >> 1);
  return (uint32_t)min(max(t, 0), M);
}
__device__ inline const uint32_t* dered_base(const SearchArgs& a, int32_t g) {
  return reinterpret_cast<const uint32_t*>(a.ws + a.dered_off) + (int64_t)g * a.dered_nb;
}
// Sample j of a trial's searched series.
__device__ inline uint32_t searched(const SearchArgs& a, const SearchRange& R,
                                    const uint32_t* base, const uint32_t* row, int64_t j) {
  const uint32_t y = row[j];
  return a.dered_shift ? dered(y, base[j >> a.dered_shift], R.full_scale) : y;
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* p, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0ull;
}

__global__ __launch_bounds__(kThreads) void k_cells(SearchArgs a) {
  extern __shared__ uint32_t sm[];  // kSub + w_max entries
  __shared__ unsigned long long red[kThreads / 64];
  __shared__ unsigned long long run_best[SDD_MAX_WIDTHS];
  __shared__ uint32_t scan_tmp[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int32_t g = blockIdx.x;
  const int r = find_range(a, g);
  const SearchRange& R = a.r[r];
  const int32_t i = g - R.dm_offset;
  const uint32_t* row = R.plane + (int64_t)i * R.pitch;
  const uint32_t* dbase = dered_base(a, g);
  Moments* mom = reinterpret_cast<Moments*>(a.ws + a.moments_off);
  CellKey* cres = reinterpret_cast<CellKey*>(a.ws + a.cellres_off);
  unsigned long long s1 = 0, s2 = 0;
  for (int32_t cell = blockIdx.y; cell < R.ncells; cell += gridDim.y) {
    const int64_t jb = (int64_t)cell * a.cand_block;
    const int64_t je = min(jb + (int64_t)a.cand_block, R.n_owned);
    if (tid < a.nwidths) run_best[tid] = 0ull;
    for (int64_t s0 = jb; s0 < je; s0 += kSub) {
      const int cnt = (int)min((int64_t)kSub, je - s0);
      const int len = cnt + a.w_max - 1;
      __syncthreads();  // previous users of sm / run_best init
      for (int k = tid; k < len; k += kThreads) sm[k] = searched(a, R, dbase, row, s0 + k);
      __syncthreads();
      for (int k = tid; k < cnt; k += kThreads) {
        unsigned long long v = sm[k];
        s1 += v;
        s2 += v * v;
      }
      // in-place exclusive prefix over sm[0, len), sm[len] = total (mod 2^32)
      const int per = (len + kThreads - 1) / kThreads;
      const int k0 = min(tid * per, len), k1 = min(k0 + per, len);
      uint32_t part = 0;
      for (int k = k0; k < k1; ++k) part += sm[k];
      uint32_t total;
      uint32_t off = block_exclusive_scan<uint32_t>(part, scan_tmp, &total);
      for (int k = k0; k < k1; ++k) {
        uint32_t v = sm[k];
        sm[k] = off;
        off += v;
      }
      if (tid == 0) sm[len] = total;
      __syncthreads();
      for (int k = 0; k < a.nwidths; ++k) {
        const int w = a.widths[k];
        unsigned long long key = 0ull;
        for (int q = tid; q < cnt; q += kThreads) {
          const uint32_t b = sm[q + w] - sm[q];
          const uint32_t jr = (uint32_t)(s0 - jb + q);
          const unsigned long long kk = ((unsigned long long)b << 32) | (uint32_t)(~jr);
          key = kk > key ? kk : key;
        }
        key = wave_max_u64(key);
        if (lane == 0) red[wid] = key;
        __syncthreads();
        if (tid == 0) {
          unsigned long long m = run_best[k];
          for (int w2 = 0; w2 < kThreads / 64; ++w2) m = red[w2] > m ? red[w2] : m;
          run_best[k] = m;
        }
        __syncthreads();
      }
    }
    __syncthreads();
    if (tid < a.nwidths) cres[(R.cell_base + (int64_t)i * R.ncells + cell) * a.nwidths + tid] =
        run_best[tid];
  }
  // exact moments of this block's owned samples
  s1 = wave_sum_u64(s1);
  s2 = wave_sum_u64(s2);
  __shared__ unsigned long long m1[kThreads / 64], m2[kThreads / 64];
  if (lane == 0) {
    m1[wid] = s1;
    m2[wid] = s2;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long t1 = 0, t2 = 0;
    for (int w2 = 0; w2 < kThreads / 64; ++w2) {
      t1 += m1[w2];
      t2 += m2[w2];
    }
    atomicAdd(&mom[g].s1, t1);
    atomicAdd(&mom[g].s2, t2);
  }
}

constexpr int kSeg = 1024;         // owned starts per wavefront
constexpr int kSegHaloMax = 1024;  // largest halo (w_max - 1, rounded up to 16)

// 16 consecutive plane samples from index j (a multiple of 16); zero at and
// past cols. Rows are 16-byte aligned (checked on the host).
__device__ inline void load16(const uint32_t* row, int64_t j, int64_t cols, uint32_t (&y)[16]) {
  if (j + 16 <= cols) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 v = *reinterpret_cast<const uint4*>(row + j + 4 * q);
      y[4 * q] = v.x;
      y[4 * q + 1] = v.y;
      y[4 * q + 2] = v.z;
      y[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 16; ++t) y[t] = j + t < cols ? row[j + t] : 0u;
  }
}

// DPP lane moves within a wavefront (VALU, no LDS): row_shr:n shifts by n
// lanes inside each row of 16 (lanes without a source read 0);
// row_bcast:15 / :31 pass lane 15 of each row / lane 31 to the following
// rows selected by the row mask.
template <int CTRL, int ROWS>
__device__ inline uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes (wrap-around uint32).
__device__ inline uint32_t wave_incl_sum(uint32_t v) {
  v += dpp<0x111, 0xf>(v);  // row_shr:1
  v += dpp<0x112, 0xf>(v);  // row_shr:2
  v += dpp<0x114, 0xf>(v);  // row_shr:4
  v += dpp<0x118, 0xf>(v);  // row_shr:8
  v += dpp<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Maximum over the 64 lanes, returned to every lane.
__device__ inline uint32_t wave_max_u32(uint32_t v) {
  uint32_t t;
  t = dpp<0x111, 0xf>(v); v = t > v ? t : v;
  t = dpp<0x112, 0xf>(v); v = t > v ? t : v;
  t = dpp<0x114, 0xf>(v); v = t > v ? t : v;
  t = dpp<0x118, 0xf>(v); v = t > v ? t : v;
  t = dpp<0x142, 0xa>(v); v = t > v ? t : v;
  t = dpp<0x143, 0xc>(v); v = t > v ? t : v;
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Exclusive prefix of 16 values per lane over the wavefront: e[t] = carry +
// sum of all earlier values; returns the wavefront total (wrap-around uint32).
__device__ inline uint32_t wave_prefix16(const uint32_t (&y)[16], uint32_t carry, uint32_t (&e)[16]) {
  uint32_t run = 0;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    e[t] = run;
    run += y[t];
  }
  const uint32_t inc = wave_incl_sum(run);
  const uint32_t off = carry + inc - run;
#pragma unroll
  for (int t = 0; t < 16; ++t) e[t] += off;
  return (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
}

// E[16 l + t + w] for t < 16: aligned 128-bit LDS reads when w % 4 == 0.
__device__ inline void read_shifted(const uint32_t* E, int lane, int w, uint32_t (&v)[16]) {
  const uint32_t* p = E + 16 * lane + w;
  if ((w & 3) == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 u = *reinterpret_cast<const uint4*>(p + 4 * q);
      v[4 * q] = u.x;
      v[4 * q + 1] = u.y;
      v[4 * q + 2] = u.z;
      v[4 * q + 3] = u.w;
    }
  } else if ((w & 1) == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint2 u = *reinterpret_cast<const uint2*>(p + 2 * q);
      v[2 * q] = u.x;
      v[2 * q + 1] = u.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 16; ++t) v[t] = p[t];
  }
}

// NARROW: every boxcar sum is below 2^28, so (B << 4) | (15 - t) orders by
// sum, then by earlier start, and one v_max per start keeps both.
// DERED: the lane's 16 samples lie in one de-reddening block (D >= 64).
template <bool NARROW, bool DERED>
__global__ __launch_bounds__(64) void k_seg(SearchArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t E[];  // kSeg + H + 4
  const int lane = threadIdx.x;
  const int32_t g = blockIdx.x;
  const int r = find_range(a, g);
  const SearchRange& R = a.r[r];
  const int32_t i = g - R.dm_offset;
  const int64_t n = R.n_owned;
  const int64_t cols = n + a.w_max - 1;
  const int32_t nseg = (int32_t)((n + kSeg - 1) / kSeg);
  const uint32_t* row = R.plane + (int64_t)i * R.pitch;
  const uint32_t* dbase = dered_base(a, g);
  const int32_t H = (a.w_max - 1 + 15) & ~15;  // halo samples
  const int32_t segs_per_cell = a.cand_block / kSeg;
  CellKey* cres = reinterpret_cast<CellKey*>(a.ws + a.cellres_off);
  // lane k holds width k: the width loop reads it with v_readlane instead of
  // a scalar load (whose wait would also drain the LDS reads)
  const int32_t wlane = lane < a.nwidths ? a.widths[lane] : 0;
  const int32_t nwidths = a.nwidths;
  const int64_t cres_row = (R.cell_base + (int64_t)i * R.ncells) * nwidths;
  unsigned long long s1 = 0, s2 = 0;
  for (int32_t seg = blockIdx.y; seg < nseg; seg += gridDim.y) {
    const int64_t j0 = (int64_t)seg * kSeg;
    const int64_t jl = j0 + 16 * lane;  // this lane's first start
    const bool full = j0 + kSeg <= n;
    uint32_t y[16], e[16];
    load16(row, jl, cols, y);
    if constexpr (DERED) {
      if (jl < cols) {
        const uint32_t b = dbase[jl >> a.dered_shift];
#pragma unroll
        for (int t = 0; t < 16; ++t) y[t] = dered(y[t], b, R.full_scale);
      }
    }
    if (full || jl + 16 <= n) {
      if constexpr (NARROW) {
        // samples are below 2^28 / w_max <= 2^28: 16 of them fit 32 bits
        uint32_t p = 0;
#pragma unroll
        for (int t = 0; t < 16; ++t) p += y[t];
        s1 += p;
      } else {
#pragma unroll
        for (int t = 0; t < 16; ++t) s1 += y[t];
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) s2 += (unsigned long long)y[t] * y[t];
    } else {
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (jl + t < n) {
          s1 += y[t];
          s2 += (unsigned long long)y[t] * y[t];
        }
    }
    const uint32_t total = wave_prefix16(y, 0u, e);
    // NARROW: LDS holds 16 * P, so 16 * P[j+w] - (16 * P[j] - (15 - t)) is
    // the packed key (B << 4) | (15 - t) in one subtraction
    constexpr int SH = NARROW ? 4 : 0;
    __syncthreads();  // the previous segment's readers are done with E
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<uint4*>(E + 16 * lane + 4 * q) =
          make_uint4(e[4 * q] << SH, e[4 * q + 1] << SH, e[4 * q + 2] << SH, e[4 * q + 3] << SH);
    if (H > 0) {
      uint32_t h[16], he[16];
      const bool hl = 16 * lane < H;
      if (hl) {
        const int64_t jh = j0 + kSeg + 16 * lane;
        load16(row, jh, cols, h);
        if constexpr (DERED) {
          if (jh < cols) {
            const uint32_t b = dbase[jh >> a.dered_shift];
#pragma unroll
            for (int t = 0; t < 16; ++t) h[t] = dered(h[t], b, R.full_scale);
          }
        }
      } else
#pragma unroll
        for (int t = 0; t < 16; ++t) h[t] = 0u;
      const uint32_t htot = wave_prefix16(h, total, he);
      if (hl)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<uint4*>(E + kSeg + 16 * lane + 4 * q) =
              make_uint4(he[4 * q] << SH, he[4 * q + 1] << SH, he[4 * q + 2] << SH,
                         he[4 * q + 3] << SH);
      if (lane == 0) E[kSeg + H] = (total + htot) << SH;
    } else if (lane == 0) {
      E[kSeg] = total << SH;
    }
    if constexpr (NARROW) {
#pragma unroll
      for (int t = 0; t < 16; ++t) e[t] = (e[t] << 4) - (uint32_t)(15 - t);
    }
    __syncthreads();
    const bool lane_ok = jl < n;
    const int32_t tmax = full ? 16 : (int32_t)min<int64_t>(16, n - jl);  // valid starts of this lane
    const int32_t cell = seg / segs_per_cell;
    const int64_t cstart = (int64_t)cell * a.cand_block;
    for (int k = 0; k < nwidths; ++k) {
      const int w = __builtin_amdgcn_readlane(wlane, k);
      uint32_t v[16];
      if (w == 1) {
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] = NARROW ? (y[t] << 4) | (uint32_t)(15 - t) : y[t];
      } else {
        read_shifted(E, lane, w, v);
#pragma unroll
        for (int t = 0; t < 16; ++t) v[t] -= e[t];
      }
      uint32_t bb, bt;
      if constexpr (NARROW) {
        // v[t] is the key of start t
        uint32_t key = 0u;
        if (full) {
#pragma unroll
          for (int t = 0; t < 16; t += 2) key = max(key, max(v[t], v[t + 1]));
        } else {
#pragma unroll
          for (int t = 0; t < 16; ++t)
            if (t < tmax) key = max(key, v[t]);
        }
        bb = key >> 4;
        bt = 15u - (key & 15u);
      } else {
        bb = v[0];
        bt = 0u;
#pragma unroll
        for (int t = 1; t < 16; ++t)
          if ((full || t < tmax) && v[t] > bb) {
            bb = v[t];
            bt = (uint32_t)t;
          }
      }
      if (!lane_ok) bb = 0u;
      const uint32_t m = wave_max_u32(bb);
      const unsigned long long hit = __ballot(lane_ok && bb == m);
      const int f = __builtin_ctzll(hit);
      const uint32_t tf = (uint32_t)__builtin_amdgcn_readlane((int)bt, f);
      if (lane == 0) {
        const int64_t j = j0 + 16 * f + tf;
        const CellKey key = ((CellKey)m << 32) | (uint32_t)(~(uint32_t)(j - cstart));
        CellKey* dst = cres + cres_row + (int64_t)cell * nwidths + k;
        if (segs_per_cell == 1)
          *dst = key;
        else
          atomicMax(dst, key);
      }
    }
  }
  s1 = wave_sum_u64(s1);
  s2 = wave_sum_u64(s2);
  if (lane == 0) {
    Moments* mom = reinterpret_cast<Moments*>(a.ws + a.moments_off);
    atomicAdd(&mom[g].s1, s1);
    atomicAdd(&mom[g].s2, s2);
  }
}

// Number of window samples <= v over the wavefront (absent ones are all-ones).
template <int E>
__device__ inline int64_t count_le(const uint32_t (&x)[E], uint32_t v) {
  int64_t c = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) c += __popcll(__ballot(x[e] <= v));
  return c;
}

// Baselines of one trial's de-reddening blocks: block k gets the lower median
// of the samples of blocks k-h..k+h (clipped to the L = N_r + w_max - 1
// columns). Each wavefront takes a run of consecutive blocks; the window of
// a block sits in registers (lane l holds samples lo + 64 e + l, e < E;
// absent ones read all-ones, above any sample), and a bisection on the value
// counts the samples <= mid with ballots. The first block of a run bisects
// between the window's minimum and maximum; the next ones first test a
// bracket [prev - b, prev + b] around the previous baseline (two counts; b
// twice the last change plus 16, at most 1024) and bisect inside it, or on
// the side the tests point to. Exact: the
// result is the smallest v with more than rank samples <= v, a sample of the
// window, whatever bracket is tried.
template <int E>
__global__ __launch_bounds__(256) void k_dered_base(SearchArgs a) {
  const int32_t g = blockIdx.x;
  const int r = find_range(a, g);
  const SearchRange& R = a.r[r];
  const uint32_t* row = R.plane + (int64_t)(g - R.dm_offset) * R.pitch;
  const int64_t L = R.n_owned + a.w_max - 1;
  const int sh = a.dered_shift, h = a.dered_half;
  const int64_t nb = (L + (1 << sh) - 1) >> sh;
  uint32_t* base = reinterpret_cast<uint32_t*>(a.ws + a.dered_off) + (int64_t)g * a.dered_nb;
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.y * 4;
  const int64_t run = (nb + waves - 1) / waves;
  const int64_t kb = ((int64_t)blockIdx.y * 4 + (threadIdx.x >> 6)) * run;
  const int64_t ke = min<int64_t>(nb, kb + run);
  uint32_t prev = 0, bw = 128;
  for (int64_t k = kb; k < ke; ++k) {
    const int64_t lo = max<int64_t>(0, (k - h) << sh);
    const int64_t hi = min<int64_t>(L, (k + h + 1) << sh);
    uint32_t x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t j = lo + 64 * e + lane;
      x[e] = j < hi ? row[j] : 0xffffffffu;
    }
    const int64_t rank = (hi - lo - 1) / 2;
    // samples are below 2^30: prev + bw cannot wrap
    bool full = k == kb;
    uint32_t vlo = 0, vhi = 0;
    bool need_min = false, need_max = false;
    if (!full) {
      const uint32_t blo = prev > bw ? prev - bw : 0u;
      const uint32_t bhi = prev + bw;
      if (count_le(x, bhi) <= rank) {  // the median lies above the bracket
        vlo = bhi + 1;
        need_max = true;
      } else if (blo > 0 && count_le(x, blo - 1) > rank) {  // below it
        vhi = blo - 1;
        need_min = true;
      } else {
        vlo = blo;
        vhi = bhi;
      }
    }
    if (full || need_min || need_max) {
      uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (lo + 64 * e + lane < hi) {
          mn = min(mn, x[e]);
          mx = max(mx, x[e]);
        }
      mn = ~wave_max_u32(~mn);
      mx = wave_max_u32(mx);
      if (full || need_min) vlo = mn;
      if (full || need_max) vhi = mx;
    }
    while (vlo < vhi) {
      const uint32_t mid = vlo + (vhi - vlo) / 2;
      if (count_le(x, mid) > rank)
        vhi = mid;
      else
        vlo = mid + 1;
    }
    if (!full) bw = min(1024u, 2u * (vlo > prev ? vlo - prev : prev - vlo) + 16u);
    prev = vlo;
    if (lane == 0) base[k] = vlo;
  }
}

// true if (s, j, w) comes before (s2, j2, w2): higher S/N, then smaller j,
// then smaller w.
__device__ inline bool better(double s, int64_t j, int w, double s2, int64_t j2, int w2) {
  if (s != s2) return s > s2;
  if (j != j2) return j < j2;
  return w < w2;
}

// mu = S1/n, sigma = sqrt(n*S2 - S1^2)/n with the numerator formed exactly (128-bit).
__device__ inline void mean_sigma_exact(uint64_t n, uint64_t s1, uint64_t s2, double* mu,
                                        double* sigma) {
  const uint64_t p_lo = n * s2, p_hi = __umul64hi(n, s2);
  const uint64_t q_lo = s1 * s1, q_hi = __umul64hi(s1, s1);
  const uint64_t d_lo = p_lo - q_lo;
  const uint64_t d_hi = p_hi - q_hi - (p_lo < q_lo ? 1ull : 0ull);
  *mu = (double)s1 / (double)n;
  *sigma = 0.0;
  if (d_hi != 0 || d_lo != 0) {
    const double dd = (double)d_hi * 18446744073709551616.0 + (double)d_lo;
    *sigma = sqrt(dd) / (double)n;
  }
}

// ---- robust noise statistics (SDD_STATS_CLIPPED, SDD_STATS_MEDIAN_MAD) ----
struct Robust {
  double mu, sigma;
  unsigned long long cnt, s1, s2, pad;
};

// Plain mean and sigma of every trial as the clipping's starting point.
__global__ __launch_bounds__(256) void k_robust_init(SearchArgs a) {
  const int32_t g = blockIdx.x * 256 + threadIdx.x;
  if (g >= a.ndm_total) return;
  const Moments m = reinterpret_cast<const Moments*>(a.ws + a.moments_off)[g];
  Robust* rb = reinterpret_cast<Robust*>(a.ws + a.robust_off) + g;
  const uint64_t n = (uint64_t)a.r[find_range(a, g)].n_owned;
  double mu, sigma;
  mean_sigma_exact(n, m.s1, m.s2, &mu, &sigma);
  rb->mu = mu;
  rb->sigma = sigma;
  rb->cnt = rb->s1 = rb->s2 = 0ull;
}

// One clipping pass: exact moments of the owned samples with
// |y - mu| <= k * sigma; blockIdx.y strides over the row.
__global__ __launch_bounds__(256) void k_clip_acc(SearchArgs a) {
  __shared__ unsigned long long red[3][4];
  const int32_t g = blockIdx.x;
  const int r = find_range(a, g);
  const SearchRange& R = a.r[r];
  const uint32_t* row = R.plane + (int64_t)(g - R.dm_offset) * R.pitch;
  const uint32_t* dbase = dered_base(a, g);
  Robust* rb = reinterpret_cast<Robust*>(a.ws + a.robust_off) + g;
  const double mu = rb->mu, lim = a.clip_k * rb->sigma;
  unsigned long long c = 0, s1 = 0, s2 = 0;
  for (int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x; j < R.n_owned;
       j += (int64_t)gridDim.y * 256) {
    const uint32_t y = searched(a, R, dbase, row, j);
    if (fabs((double)y - mu) <= lim) {
      c += 1;
      s1 += y;
      s2 += (unsigned long long)y * y;
    }
  }
  c = wave_sum_u64(c);
  s1 = wave_sum_u64(s1);
  s2 = wave_sum_u64(s2);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = c;
    red[1][w] = s1;
    red[2][w] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&rb->cnt, red[0][0] + red[0][1] + red[0][2] + red[0][3]);
    atomicAdd(&rb->s1, red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    atomicAdd(&rb->s2, red[2][0] + red[2][1] + red[2][2] + red[2][3]);
  }
}

// New mu, sigma from the kept samples (unchanged when none was kept).
__global__ __launch_bounds__(256) void k_clip_update(SearchArgs a) {
  const int32_t g = blockIdx.x * 256 + threadIdx.x;
  if (g >= a.ndm_total) return;
  Robust* rb = reinterpret_cast<Robust*>(a.ws + a.robust_off) + g;
  if (rb->cnt > 0) {
    double mu, sigma;
    mean_sigma_exact(rb->cnt, rb->s1, rb->s2, &mu, &sigma);
    rb->mu = mu;
    rb->sigma = sigma;
  }
  rb->cnt = rb->s1 = rb->s2 = 0ull;
}

// Lower median of the owned samples (what == 0) or of |y - median| (what ==
// 1) of one trial per workgroup: radix selection, 11 bits per pass.
__global__ __launch_bounds__(1024) void k_row_select(SearchArgs a, int what, int passes) {
  __shared__ uint32_t hist[2048];
  __shared__ uint32_t s_prefix;
  __shared__ int64_t s_k;
  const int32_t g = blockIdx.x;
  const int r = find_range(a, g);
  const SearchRange& R = a.r[r];
  const uint32_t* row = R.plane + (int64_t)(g - R.dm_offset) * R.pitch;
  const uint32_t* dbase = dered_base(a, g);
  Robust* rb = reinterpret_cast<Robust*>(a.ws + a.robust_off) + g;
  const int64_t n = R.n_owned;
  const int64_t med = what ? (int64_t)rb->mu : 0;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_prefix = 0u;
    s_k = (n - 1) / 2;
  }
  uint32_t hmask = 0u;
  for (int ps = passes - 1; ps >= 0; --ps) {
    for (int b = tid; b < 2048; b += 1024) hist[b] = 0u;
    __syncthreads();
    const uint32_t prefix = s_prefix;
    const int sh = 11 * ps;
    for (int64_t j = tid; j < n; j += 1024) {
      int64_t v = searched(a, R, dbase, row, j);
      if (what) v = v > med ? v - med : med - v;
      const uint32_t u = (uint32_t)v;
      if ((u & hmask) == prefix) atomicAdd(&hist[(u >> sh) & 2047u], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      int64_t kk = s_k;
      int bin = 0;
      for (; bin < 2047; ++bin) {
        if (kk < (int64_t)hist[bin]) break;
        kk -= hist[bin];
      }
      s_k = kk;
      s_prefix = prefix | ((uint32_t)bin << sh);
    }
    __syncthreads();
    hmask |= 2047u << sh;
  }
  if (tid == 0) {
    if (what)
      rb->sigma = 1.4826 * (double)s_prefix;
    else
      rb->mu = (double)s_prefix;
  }
}

__global__ __launch_bounds__(kThreads) void k_rows(SearchArgs a) {
  __shared__ double rs[kThreads];
  __shared__ int64_t rj[kThreads];
  __shared__ int rw[kThreads];
  __shared__ int rc[kThreads];
  const int tid = threadIdx.x;
  const int32_t g = blockIdx.x;
  const int r = find_range(a, g);
  const SearchRange& R = a.r[r];
  const int32_t i = g - R.dm_offset;
  const Moments m = reinterpret_cast<const Moments*>(a.ws + a.moments_off)[g];
  const CellKey* cres = reinterpret_cast<const CellKey*>(a.ws + a.cellres_off);
  CellBest* cbest = reinterpret_cast<CellBest*>(a.ws + a.cellbest_off);
  const uint64_t n = (uint64_t)R.n_owned;
  double mu, sigma;
  if (a.stats_mode == SDD_STATS_MOMENTS) {
    mean_sigma_exact(n, m.s1, m.s2, &mu, &sigma);
  } else {
    const Robust* rb = reinterpret_cast<const Robust*>(a.ws + a.robust_off) + g;
    mu = rb->mu;
    sigma = rb->sigma;
  }
  if (tid == 0 && a.stats) {
    sdd_dm_stats st;
    st.n = (int64_t)n;
    st.s1 = m.s1;
    st.s2 = m.s2;
    st.mean = mu;
    st.std = sigma;
    a.stats[g] = st;
  }
  double bs = -INFINITY;
  int64_t bj = 0;
  int bw = 0;
  int cnt = 0;
  const double thr = (double)a.threshold;
  for (int32_t c = tid; c < R.ncells; c += kThreads) {
    const int64_t cidx = R.cell_base + (int64_t)i * R.ncells + c;
    const CellKey* cr = cres + cidx * a.nwidths;
    const int64_t cstart = (int64_t)c * a.cand_block;
    double cs;
    int64_t cj;
    int cw;
    if (sigma == 0.0) {
      cs = 0.0;
      cj = (int64_t)c * a.cand_block;
      cw = a.widths[0];
    } else {
      cs = -INFINITY;
      cj = 0;
      cw = 0;
      for (int k = 0; k < a.nwidths; ++k) {
        const int w = a.widths[k];
        const CellKey key = cr[k];
        const uint32_t b = (uint32_t)(key >> 32);
        const int64_t j = cstart + (int64_t)(~(uint32_t)key);
        const double s = ((double)b - (double)w * mu) / (sigma * sqrt((double)w));
        if (better(s, j, w, cs, cj, cw)) {
          cs = s;
          cj = j;
          cw = w;
        }
      }
    }
    const bool flag = sigma > 0.0 && cs > thr;
    CellBest cb;
    cb.snr = cs;
    cb.j = (int32_t)cj;
    cb.wf = (uint32_t)cw | (flag ? 0x80000000u : 0u);
    cbest[cidx] = cb;
    cnt += flag ? 1 : 0;
    if (better(cs, cj, cw, bs, bj, bw)) {
      bs = cs;
      bj = cj;
      bw = cw;
    }
  }
  rs[tid] = bs;
  rj[tid] = bj;
  rw[tid] = bw;
  rc[tid] = cnt;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
      if (better(rs[tid + h], rj[tid + h], rw[tid + h], rs[tid], rj[tid], rw[tid])) {
        rs[tid] = rs[tid + h];
        rj[tid] = rj[tid + h];
        rw[tid] = rw[tid + h];
      }
      rc[tid] += rc[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    sdd_dm_best b;
    b.snr = (float)rs[0];
    b.width = rw[0];
    b.sample = rj[0];
    a.best[g] = b;
    reinterpret_cast<int32_t*>(a.ws + a.rowcnt_off)[g] = rc[0];
  }
}

__global__ __launch_bounds__(1024) void k_scan(SearchArgs a) {
  __shared__ int32_t tmp[16];
  const int32_t* cnt = reinterpret_cast<const int32_t*>(a.ws + a.rowcnt_off);
  int32_t* off = reinterpret_cast<int32_t*>(a.ws + a.rowoff_off);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int32_t carry = 0;
  for (int32_t base = 0; base < a.ndm_total; base += 1024) {
    const int32_t g = base + tid;
    const int32_t v = g < a.ndm_total ? cnt[g] : 0;
    int32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
      int32_t t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    if (lane == 63) tmp[wid] = inc;
    __syncthreads();
    int32_t woff = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wid) woff += tmp[w];
      tot += tmp[w];
    }
    if (g < a.ndm_total) off[g] = carry + woff + inc - v;
    carry += tot;
    __syncthreads();
  }
  if (tid == 0) {
    off[a.ndm_total] = carry;
    *a.ncand = carry;
  }
}

__global__ __launch_bounds__(kThreads) void k_compact(SearchArgs a) {
  __shared__ int32_t tmp[kThreads / 64];
  const int tid = threadIdx.x;
  const int32_t g = blockIdx.x;
  const int r = find_range(a, g);
  const SearchRange& R = a.r[r];
  const int32_t i = g - R.dm_offset;
  const CellBest* cbest = reinterpret_cast<const CellBest*>(a.ws + a.cellbest_off);
  int32_t base = reinterpret_cast<const int32_t*>(a.ws + a.rowoff_off)[g];
  for (int32_t c0 = 0; c0 < R.ncells; c0 += kThreads) {
    const int32_t c = c0 + tid;
    CellBest cb{};
    bool flag = false;
    if (c < R.ncells) {
      cb = cbest[R.cell_base + (int64_t)i * R.ncells + c];
      flag = (cb.wf & 0x80000000u) != 0;
    }
    int32_t total;
    const int32_t ex = block_exclusive_scan<int32_t>(flag ? 1 : 0, tmp, &total);
    const int32_t at = base + ex;
    if (flag && at < a.cap) {
      sdd_candidate o;
      o.range = r;
      o.dm_index = i;
      o.sample = cb.j;
      o.width = (int32_t)(cb.wf & 0x7fffffffu);
      o.snr = (float)cb.snr;
      a.cands[at] = o;
    }
    base += total;
  }
}

}  // namespace

hipError_t launch_search(const SearchArgs& a, hipStream_t s) {
  if (a.ndm_total <= 0) return hipSuccess;
  const int64_t nm = 2 * (int64_t)a.ndm_total;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<unsigned long long*>(a.ws + a.moments_off), nm);
  if (a.dered_shift) {
    int64_t nb = 0;
    for (int r = 0; r < a.nranges; ++r)
      nb = std::max<int64_t>(nb, (a.r[r].n_owned + a.w_max - 1 + (1 << a.dered_shift) - 1) >>
                                     a.dered_shift);
    if (nb > a.dered_nb) return hipErrorInvalidValue;
    // runs of about 16 consecutive blocks per wavefront, 4 wavefronts per workgroup
    const dim3 gr((unsigned)a.ndm_total, (unsigned)std::max<int64_t>(1, std::min<int64_t>(
                                             (nb + 63) / 64, 65535)));
    const int ne = a.dered_elems;
    if (ne <= 4)
      hipLaunchKernelGGL(k_dered_base<4>, gr, dim3(256), 0, s, a);
    else if (ne <= 8)
      hipLaunchKernelGGL(k_dered_base<8>, gr, dim3(256), 0, s, a);
    else if (ne <= 12)
      hipLaunchKernelGGL(k_dered_base<12>, gr, dim3(256), 0, s, a);
    else if (ne <= 16)
      hipLaunchKernelGGL(k_dered_base<16>, gr, dim3(256), 0, s, a);
    else if (ne <= 20)
      hipLaunchKernelGGL(k_dered_base<20>, gr, dim3(256), 0, s, a);
    else if (ne <= 24)
      hipLaunchKernelGGL(k_dered_base<24>, gr, dim3(256), 0, s, a);
    else if (ne <= 32)
      hipLaunchKernelGGL(k_dered_base<32>, gr, dim3(256), 0, s, a);
    else if (ne <= 48)
      hipLaunchKernelGGL(k_dered_base<48>, gr, dim3(256), 0, s, a);
    else if (ne <= 64)
      hipLaunchKernelGGL(k_dered_base<64>, gr, dim3(256), 0, s, a);
    else
      return hipErrorInvalidValue;
  }
  const int32_t halo = (a.w_max - 1 + 15) & ~15;
  bool seg_ok = a.nwidths > 0 && a.cand_block % kSeg == 0 && halo <= kSegHaloMax;
  int64_t max_owned = 0;
  for (int r = 0; r < a.nranges; ++r) {
    seg_ok = seg_ok && (uintptr_t)a.r[r].plane % 16 == 0 && a.r[r].pitch % 4 == 0;
    max_owned = std::max(max_owned, a.r[r].n_owned);
  }
  if (seg_ok) {
    const int64_t nseg = (max_owned + kSeg - 1) / kSeg;
    if (a.cand_block > kSeg) {
      // cells of several segments combine their keys with atomic max
      int64_t ncell = 0;
      for (int r = 0; r < a.nranges; ++r) ncell += (int64_t)a.r[r].ndm * a.r[r].ncells;
      const int64_t nk = ncell * a.nwidths;
      hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s,
                         reinterpret_cast<unsigned long long*>(a.ws + a.cellres_off), nk);
    }
    // a few segments per workgroup (a grid-stride loop) amortize its set-up
    const int64_t per_wg = std::max<int64_t>(1, std::min<int64_t>(4, nseg / 64));
    const unsigned gy =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>((nseg + per_wg - 1) / per_wg, 65535));
    const size_t lds = (size_t)(kSeg + halo + 4) * sizeof(uint32_t);
    const dim3 gr((unsigned)a.ndm_total, gy);
    const bool narrow = a.max_boxcar < ((int64_t)1 << 28);
    if (a.dered_shift) {
      if (narrow)
        hipLaunchKernelGGL((k_seg<true, true>), gr, dim3(64), lds, s, a);
      else
        hipLaunchKernelGGL((k_seg<false, true>), gr, dim3(64), lds, s, a);
    } else if (narrow) {
      hipLaunchKernelGGL((k_seg<true, false>), gr, dim3(64), lds, s, a);
    } else {
      hipLaunchKernelGGL((k_seg<false, false>), gr, dim3(64), lds, s, a);
    }
  } else {
    const unsigned gy =
        (unsigned)(a.max_cells < 1 ? 1 : (a.max_cells > 65535 ? 65535 : a.max_cells));
    const size_t lds = (size_t)(kSub + a.w_max) * sizeof(uint32_t);
    hipLaunchKernelGGL(k_cells, dim3((unsigned)a.ndm_total, gy), dim3(kThreads), lds, s, a);
  }
  if (a.stats_mode == SDD_STATS_CLIPPED) {
    const dim3 gr((unsigned)((a.ndm_total + 255) / 256));
    hipLaunchKernelGGL(k_robust_init, gr, dim3(256), 0, s, a);
    for (int it = 0; it < a.clip_iters; ++it) {
      hipLaunchKernelGGL(k_clip_acc, dim3((unsigned)a.ndm_total, 16), dim3(256), 0, s, a);
      hipLaunchKernelGGL(k_clip_update, gr, dim3(256), 0, s, a);
    }
  } else if (a.stats_mode == SDD_STATS_MEDIAN_MAD) {
    int bits = 1;
    while (bits < 32 && (a.max_sample >> bits) != 0) ++bits;
    const int passes = (bits + 10) / 11;
    hipLaunchKernelGGL(k_row_select, dim3((unsigned)a.ndm_total), dim3(1024), 0, s, a, 0, passes);
    hipLaunchKernelGGL(k_row_select, dim3((unsigned)a.ndm_total), dim3(1024), 0, s, a, 1, passes);
  }
  hipLaunchKernelGGL(k_rows, dim3((unsigned)a.ndm_total), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_compact, dim3((unsigned)a.ndm_total), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace sdd
