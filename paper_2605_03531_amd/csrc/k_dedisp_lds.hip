// LDS-tiled brute-force dedispersion of uint8 channel rows (Section 3.2:
// every trial DM sums all channels along its delay curve):
//   plane[i][j] = sum_c x[c][j + delay[c][i]]
//
// One workgroup owns a tile of DT = D*WD trials x TT = 512*M*WT samples and
// walks the channels in stages of CS. For each channel it stages the window
// of input bytes every trial of the tile needs, [t0 + d(c,i0), t0 + TT +
// d(c,i_last)), in LDS twice: as loaded (copy 0) and shifted by 4 bytes
// (copy 1). A lane owns 8 consecutive samples per chunk; for trial i it reads
// 12 bytes (one 64-bit and one 32-bit LDS read, both aligned) from the copy
// that leaves the wanted 8 bytes at an offset s < 4, and v_perm both aligns
// and widens them into four pairs of 16-bit fields. v_add3 adds two channels
// into each packed accumulator; every 256 channels the packed fields are
// flushed into uint32 sums (256 * 255 < 2^16 keeps the fields exact).
//
// Wavefronts split the tile: WD groups along DM (D trials each) x WT groups
// along time (M chunks of 512 samples each). Lanes of a chunk read
// consecutive 8-byte words, so LDS reads are free of bank conflicts.
// Workgroups are ordered DM-tile-major and each XCD takes a contiguous run of
// tiles, so the concurrently running tiles of one XCD are neighbours in time
// whose input windows overlap in that XCD's L2.
#include "k_dedisp_lds.h"

namespace sdd {
namespace {

// One DT x TT tile of one job. Every thread of the workgroup calls it; it
// returns after a barrier, so the caller may reuse the LDS at once.
// ES = input element bytes: 1 (uint8 rows) or 2 (uint16 rows of a decimated
// range). A lane always owns 8 bytes of a 512-byte chunk: 8 uint8 samples
// (four 16-bit pairs after widening) or 4 uint16 samples (two pairs as read).
template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
__device__ __forceinline__ void dd_tile(const LdsArgs a, int32_t dtile, int32_t ttile,
                                        uint8_t* __restrict__ lds) {
  constexpr int NT = 64 * WD * WT;
  constexpr int DT = D * WD;
  constexpr int SPL = 8 / ES;       // samples per lane per chunk
  constexpr int CH = 64 * SPL;      // samples per 512-byte chunk
  constexpr int NPK = SPL / 2;      // packed 16-bit pairs per lane per chunk
  constexpr int TW = CH * M;        // samples per time group of waves
  constexpr int TT = TW * WT;
  const int32_t i0 = dtile * DT;
  const int64_t t0 = (int64_t)ttile * TT;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wd = wave % WD, wt = wave / WD;
  const int32_t ndm = a.ndm, nchan = a.nchan;
  const int32_t* __restrict__ dcm = a.delays;

  int32_t iw[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int32_t i = i0 + wd * D + d;
    iw[d] = i < ndm ? i : ndm - 1;
  }

  const int32_t win = a.win;            // bytes per copy, multiple of 16
  const int32_t slot = 2 * win;         // copy 0 + copy 1
  const int32_t buf = CS * slot;
  const int32_t wq = win >> 4;          // 16-byte elements per window

  uint32_t acc[D][M][NPK];
  uint32_t wide[D][M][SPL];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int m = 0; m < M; ++m) {
#pragma unroll
      for (int k = 0; k < NPK; ++k) acc[d][m][k] = 0u;
#pragma unroll
      for (int k = 0; k < SPL; ++k) wide[d][m][k] = 0u;
    }

  // ---- staging: global -> registers -> two LDS copies ----
  constexpr bool PREF2 = (F & 1) != 0;  // prefetch LDS stages two ahead
  constexpr bool WIDE = (F & 2) != 0;   // 2 x 64-bit reads instead of 64 + 32
  // window bases from delays fetched a stage earlier (no dependent global
  // load in the staging path); element and delay lane maps computed once
  constexpr bool EARLY = (F & 4) != 0;
  static_assert(!(EARLY && PREF2), "one prefetch scheme at a time");
  // the staging must hold a stage's windows at zero delay span at least
  static_assert(CS * (ES * TT + 32 * ES) <= 16 * NLD * NT, "staging too small for the tile");
  int32_t ecs[NLD], eq[NLD];
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int32_t e = tid + k * NT;
    ecs[k] = e / wq;
    eq[k] = e - ecs[k] * wq;
  }
  uint4 st[NLD];
  uint4 st2[PREF2 ? NLD : 1];
  auto load_stage = [&](int32_t cbase, uint4 (&dst)[NLD]) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int32_t e = tid + k * NT;
      const int32_t cs = e / wq;
      const int32_t q = e - cs * wq;
      const int32_t c = cbase + cs;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (cs < CS && c < nchan) {
        // byte g of channel c's row; the window starts at sample t0 + d(c,i0) & ~15
        const int64_t g = ES * (t0 + (int64_t)(dcm[(int64_t)c * ndm + i0] & ~15)) + 16 * q;
        const int64_t row_bytes = ES * a.x_len;
        const uint8_t* src = a.x + (int64_t)c * a.x_pitch * ES + g;
        if (a.aligned && g + 16 <= row_bytes) {
          v = *reinterpret_cast<const uint4*>(src);
        } else {
          uint32_t w[4] = {0u, 0u, 0u, 0u};
          for (int bb = 0; bb < 16; ++bb)
            if (g + bb < row_bytes) w[bb >> 2] |= (uint32_t)src[bb] << (8 * (bb & 3));
          v = make_uint4(w[0], w[1], w[2], w[3]);
        }
      }
      dst[k] = v;
    }
  };
  // staging with the window bases taken from a delay vector of the stage
  // (entry cs*(D+1) holds d(c, i0) of slot cs)
  auto load_stage_bases = [&](int32_t cbase, uint4 (&dst)[NLD], const int32_t* dv) {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int32_t cs = ecs[k], q = eq[k];
      const int32_t c = cbase + cs;
      const int32_t idx = (cs < CS ? cs : 0) * (D + 1);
      int32_t b0 = __shfl(dv[0], idx & 63, 64);
      if ((CS * (D + 1) + 63) / 64 > 1) {
        const int32_t b1 = __shfl(dv[((CS * (D + 1) + 63) / 64) - 1], idx & 63, 64);
        b0 = idx < 64 ? b0 : b1;
      }
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (cs < CS && c < nchan) {
        const int64_t g = ES * (t0 + (int64_t)(b0 & ~15)) + 16 * q;
        const int64_t row_bytes = ES * a.x_len;
        const uint8_t* src = a.x + (int64_t)c * a.x_pitch * ES + g;
        if (a.aligned && g + 16 <= row_bytes) {
          v = *reinterpret_cast<const uint4*>(src);
        } else {
          uint32_t w[4] = {0u, 0u, 0u, 0u};
          for (int bb = 0; bb < 16; ++bb)
            if (g + bb < row_bytes) w[bb >> 2] |= (uint32_t)src[bb] << (8 * (bb & 3));
          v = make_uint4(w[0], w[1], w[2], w[3]);
        }
      }
      dst[k] = v;
    }
  };
  auto store_stage = [&](int32_t which, const uint4 (&src)[NLD]) {
    uint8_t* base = lds + which * buf;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int32_t cs = ecs[k];
      const int32_t q = eq[k];
      if (cs < CS) {
        uint8_t* c0 = base + cs * slot + 16 * q;  // copy 0
        uint8_t* c1 = c0 + win;                   // copy 1: byte j holds window byte j + 4
        *reinterpret_cast<uint4*>(c0) = src[k];
        if (q > 0) *reinterpret_cast<uint32_t*>(c1 - 4) = src[k].x;
        *reinterpret_cast<uint2*>(c1) = make_uint2(src[k].y, src[k].z);
        *reinterpret_cast<uint32_t*>(c1 + 8) = src[k].w;
      }
    }
  };

  auto flush = [&]() {
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < NPK; ++k) {
          wide[d][m][2 * k] += acc[d][m][k] & 0xffffu;
          wide[d][m][2 * k + 1] += acc[d][m][k] >> 16;
          acc[d][m][k] = 0u;
        }
  };

  // Delays of the next stage travel with its data: lane k < CS*(D+1) loads
  // one entry (slot k/(D+1); entry 0 = the tile's first trial, entry 1+d =
  // this wavefront's trial d) through the vector memory path, so the compute
  // loop holds no scalar-memory waits that would also drain its LDS reads.
  // A channel past nchan gets delay 0 and an all-zero window.
  constexpr int DE = D + 1;
  constexpr int NDV = (CS * DE + 63) / 64;  // VGPRs holding one stage's delays
  int32_t dl_cs[NDV], dl_i[NDV];
  bool dl_e0[NDV];
#pragma unroll
  for (int v = 0; v < NDV; ++v) {
    const int32_t k = 64 * v + lane;
    const int32_t cs = k / DE, e = k - cs * DE;
    int32_t i = e == 0 ? i0 : i0 + wd * D + e - 1;
    dl_cs[v] = k < CS * DE ? cs : CS;
    dl_i[v] = i < ndm ? i : ndm - 1;
    dl_e0[v] = e == 0;
  }
  // Entry 0 of a slot keeps the raw delay d(c, i0) (the window base); entry
  // 1+d holds the packed read position of trial d: bits 0-19 the LDS byte
  // offset of its 8-byte word inside the slot (copy 1 when the offset within
  // the word is >= 4), bits 20-21 the remaining byte shift. Computing it here,
  // once per stage for all entries across the lanes, keeps the per-trial work
  // in the loop to one v_readlane and a few scalar operations.
  auto load_delays = [&](int32_t cbase, int32_t (&out)[NDV]) {
#pragma unroll
    for (int v = 0; v < NDV; ++v) {
      const int32_t c = cbase + dl_cs[v];
      const bool ok = dl_cs[v] < CS && c < nchan;
      const int32_t* row = dcm + (int64_t)(ok ? c : 0) * ndm;
      const int32_t dv = ok ? row[dl_i[v]] : 0;
      const int32_t d0 = ok ? row[i0] : 0;
      const int32_t o = ES * (dv - (d0 & ~15));
      const int32_t ad = (o & ~7) + ((o & 4) ? win : 0);
      out[v] = dl_e0[v] ? d0 : (ad | ((o & 3) << 20));
    }
  };
  // entry k of the current stage, as a wave-uniform scalar
#define SDD_DELAY(k) __builtin_amdgcn_readlane(dcur[(k) / 64], (k) % 64)

  const int32_t nstages = (nchan + CS - 1) / CS;
  const int32_t lane_off = 8 * lane + ES * TW * wt;  // bytes
  const int32_t flush_every = ES == 1 ? 256 : a.flush;
  int32_t dnext[NDV];
  int32_t dnext2[(PREF2 || EARLY) ? NDV : 1];
  if constexpr (EARLY) {
    load_delays(0, dnext);
    load_stage_bases(0, st, dnext);
    if (nstages > 1) load_delays(CS, dnext2);
  } else {
    load_stage(0, st);
    load_delays(0, dnext);
  }
  store_stage(0, st);
  if constexpr (PREF2) {
    if (nstages > 1) {
      load_stage(CS, st);
      load_delays(CS, dnext2);
    }
  }
  __syncthreads();
  for (int32_t s = 0; s < nstages; ++s) {
    const int32_t cbase = s * CS;
    int32_t dcur[NDV];
#pragma unroll
    for (int v = 0; v < NDV; ++v) dcur[v] = dnext[v];
    if constexpr (EARLY) {
      // stage s+1's delays arrived a stage ago: stage its data now, fetch
      // the delays of stage s+2
      if (s + 1 < nstages) load_stage_bases(cbase + CS, st, dnext2);
#pragma unroll
      for (int v = 0; v < NDV; ++v) dnext[v] = dnext2[v];
      if (s + 2 < nstages) load_delays(cbase + 2 * CS, dnext2);
    } else if constexpr (PREF2) {
      // stage s+1 is in st (loaded one stage ago); fetch stage s+2
      if (s + 2 < nstages) {
        load_stage(cbase + 2 * CS, st2);
        int32_t dtmp[NDV];
        load_delays(cbase + 2 * CS, dtmp);
#pragma unroll
        for (int v = 0; v < NDV; ++v) {
          dnext[v] = dnext2[v];
          dnext2[v] = dtmp[v];
        }
      } else {
#pragma unroll
        for (int v = 0; v < NDV; ++v) dnext[v] = dnext2[v];
      }
    } else if (s + 1 < nstages) {
      load_stage(cbase + CS, st);
      load_delays(cbase + CS, dnext);
    }
    const uint8_t* bufp = lds + (s & 1) * buf + lane_off;
#pragma unroll
    for (int cc = 0; cc < CS; cc += 2) {
      const uint8_t* slotA = bufp + cc * slot;
      const uint8_t* slotB = slotA + slot;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const uint32_t wA = (uint32_t)SDD_DELAY(cc * DE + 1 + d);
        const uint32_t wB = (uint32_t)SDD_DELAY((cc + 1) * DE + 1 + d);
        const int32_t adA = (int32_t)(wA & 0xfffffu);
        const int32_t adB = (int32_t)(wB & 0xfffffu);
        const uint32_t rA = wA >> 20, rB = wB >> 20;
        // v_perm selectors: bytes r, r+1 (and r+2, r+3) into 16-bit fields for
        // uint8 input; bytes r..r+3 in order for uint16 input
        const uint32_t sA0 = ES == 1 ? 0x0c010c00u + rA * 0x00010001u : 0x03020100u + rA * 0x01010101u;
        const uint32_t sB0 = ES == 1 ? 0x0c010c00u + rB * 0x00010001u : 0x03020100u + rB * 0x01010101u;
        const uint32_t sA2 = sA0 + 0x00020002u;
        const uint32_t sB2 = sB0 + 0x00020002u;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const uint8_t* pA = slotA + adA + 512 * m;
          const uint8_t* pB = slotB + adB + 512 * m;
          const uint2 a01 = *reinterpret_cast<const uint2*>(pA);
          const uint2 b01 = *reinterpret_cast<const uint2*>(pB);
          uint32_t a2, b2;
          if constexpr (WIDE) {
            const uint2 a23 = *reinterpret_cast<const uint2*>(pA + 8);
            const uint2 b23 = *reinterpret_cast<const uint2*>(pB + 8);
            // keep the full 64-bit reads (conflict-free at an 8-byte lane stride)
            asm volatile("" ::"v"(a23.y), "v"(b23.y));
            a2 = a23.x;
            b2 = b23.x;
          } else {
            a2 = *reinterpret_cast<const uint32_t*>(pA + 8);
            b2 = *reinterpret_cast<const uint32_t*>(pB + 8);
          }
          if constexpr (ES == 1) {
            acc[d][m][0] += __builtin_amdgcn_perm(a01.y, a01.x, sA0) +
                            __builtin_amdgcn_perm(b01.y, b01.x, sB0);
            acc[d][m][1] += __builtin_amdgcn_perm(a01.y, a01.x, sA2) +
                            __builtin_amdgcn_perm(b01.y, b01.x, sB2);
            acc[d][m][2] += __builtin_amdgcn_perm(a2, a01.y, sA0) +
                            __builtin_amdgcn_perm(b2, b01.y, sB0);
            acc[d][m][3] += __builtin_amdgcn_perm(a2, a01.y, sA2) +
                            __builtin_amdgcn_perm(b2, b01.y, sB2);
          } else {
            // uint16 samples are already 16-bit fields: v_perm only aligns
            acc[d][m][0] += __builtin_amdgcn_perm(a01.y, a01.x, sA0) +
                            __builtin_amdgcn_perm(b01.y, b01.x, sB0);
            acc[d][m][1] += __builtin_amdgcn_perm(a2, a01.y, sA0) +
                            __builtin_amdgcn_perm(b2, b01.y, sB0);
          }
        }
      }
    }
    if ((cbase + CS) % flush_every == 0 || s + 1 == nstages) flush();
    if (s + 1 < nstages) store_stage((s + 1) & 1, st);
    if constexpr (PREF2) {
#pragma unroll
      for (int k = 0; k < NLD; ++k) st[k] = st2[k];
    }
    __syncthreads();
  }

#undef SDD_DELAY

  // ---- store the tile ----
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int32_t i = i0 + wd * D + d;
    if (i >= ndm) break;
    uint32_t* row = a.plane + (int64_t)i * a.plane_pitch;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int64_t j = t0 + TW * wt + CH * m + SPL * lane;
      if (j + SPL <= a.cols) {
#pragma unroll
        for (int k = 0; k < SPL; k += 4)
          *reinterpret_cast<uint4*>(row + j + k) =
              make_uint4(wide[d][m][k], wide[d][m][k + 1], wide[d][m][k + 2], wide[d][m][k + 3]);
      } else {
#pragma unroll
        for (int k = 0; k < SPL; ++k)
          if (j + k < a.cols) row[j + k] = wide[d][m][k];
      }
    }
  }
}

// Grid form: one workgroup per tile of one job, ordered DM-tile-major with a
// contiguous run of tiles per XCD (workgroups go to the 8 XCDs round-robin).
template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
__global__ __launch_bounds__(64 * WD * WT) void k_dedisp_lds(LdsArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int32_t nblk = a.n_dtiles * a.n_ttiles;
  const int32_t b = blockIdx.x;
  const int32_t full = nblk & ~7;
  const int32_t L = b < full ? (b & 7) * (full >> 3) + (b >> 3) : b;
  const int32_t dtile = L / a.n_ttiles;
  dd_tile<D, M, WD, WT, CS, NLD, F, ES>(a, dtile, L - dtile * a.n_ttiles, lds);
}

// Persistent form for a batch of jobs (beams x DM ranges with the same tile
// shape): the global tile list (job by job, DM-tile-major inside a job) is
// cut into 8 contiguous parts, one per XCD; the workgroups of an XCD take
// the tiles of its part in order from an atomic counter until it runs dry.
template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
__global__ __launch_bounds__(64 * WD * WT) void k_dedisp_lds_multi(MultiArgs m) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  __shared__ int32_t s_tile;
  const int32_t total = m.tile_base[m.njobs];
  const int xcd = blockIdx.x & 7;
  const int32_t lo = (int32_t)(((int64_t)total * xcd) >> 3);
  const int32_t hi = (int32_t)(((int64_t)total * (xcd + 1)) >> 3);
  for (;;) {
    if (threadIdx.x == 0) s_tile = lo + (int32_t)atomicAdd(&m.counters[xcd], 1u);
    __syncthreads();
    const int32_t t = s_tile;
    __syncthreads();
    if (t >= hi) break;
    int j = 0;
    while (j + 1 < m.njobs && t >= m.tile_base[j + 1]) ++j;
    const LdsArgs a = m.jobs[j];
    const int32_t L = t - m.tile_base[j];
    const int32_t dtile = L / a.n_ttiles;
    dd_tile<D, M, WD, WT, CS, NLD, F, ES>(a, dtile, L - dtile * a.n_ttiles, lds);
  }
}

__global__ void k_zero_counters(uint32_t* c) {
  if (threadIdx.x < 8) c[threadIdx.x] = 0u;
}

template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
hipError_t launch_multi(const MultiArgs& m, int32_t max_win, hipStream_t s) {
  constexpr int NT = 64 * WD * WT;
  const size_t lds = (size_t)2 * CS * 2 * max_win;
  auto kern = k_dedisp_lds_multi<D, M, WD, WT, CS, NLD, F, ES>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, lds);
  if (e != hipSuccess) return e;
  int dev = 0, ncu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  int nblk = (per_cu < 1 ? 1 : per_cu) * ncu;
  nblk = (nblk + 7) / 8 * 8;
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, m.counters);
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(NT), lds, s, m);
  return hipGetLastError();
}

template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
hipError_t launch_one(const LdsArgs& a, hipStream_t s) {
  constexpr int NT = 64 * WD * WT;
  const size_t lds = (size_t)2 * CS * 2 * a.win;
  auto kern = k_dedisp_lds<D, M, WD, WT, CS, NLD, F, ES>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const unsigned nblk = (unsigned)(a.n_dtiles * a.n_ttiles);
  hipLaunchKernelGGL(kern, dim3(nblk), dim3(NT), lds, s, a);
  return hipGetLastError();
}

}  // namespace

// The built menu, {D, M, WD, WT, CS, NLD, F}; sdd_tile carries it as
// {kind 1 + F, D, WD, WT, pairs per lane = 4*M, CS}.
#define SDD_LDS_SHAPES(X)      \
  X(2, 2, 4, 1, 4, 2, 4)       \
  X(2, 1, 4, 1, 4, 1, 4)       \
  X(4, 1, 4, 1, 4, 2, 4)       \
  X(4, 1, 2, 2, 4, 2, 4)       \
  X(2, 2, 2, 1, 4, 3, 4)       \
  X(4, 1, 2, 1, 4, 2, 4)       \
  X(4, 1, 8, 1, 4, 1, 4)       \
  X(4, 1, 4, 2, 4, 2, 4)       \
  X(2, 1, 8, 1, 4, 1, 4)       \
  X(4, 1, 16, 1, 4, 1, 4)      \
  X(4, 1, 8, 2, 4, 1, 4)       \
  X(4, 1, 8, 2, 4, 1, 0)       \
  X(4, 1, 8, 2, 4, 1, 1)       \
  X(4, 1, 8, 2, 4, 1, 6)       \
  X(8, 1, 4, 1, 8, 4, 0)

#define SDD_SHAPE_ROW(d, m, wd, wt, cs, nld, f) {d, m, wd, wt, cs, nld, f},
#define SDD_ONE_PTR(d, m, wd, wt, cs, nld, f) \
  {&launch_one<d, m, wd, wt, cs, nld, f, 1>, &launch_one<d, m, wd, wt, cs, nld, f, 2>},
#define SDD_MULTI_PTR(d, m, wd, wt, cs, nld, f) \
  {&launch_multi<d, m, wd, wt, cs, nld, f, 1>, &launch_multi<d, m, wd, wt, cs, nld, f, 2>},

const LdsShape kLdsShapes[] = {SDD_LDS_SHAPES(SDD_SHAPE_ROW)};
const int kNumLdsShapes = sizeof(kLdsShapes) / sizeof(kLdsShapes[0]);

namespace {
using OneFn = hipError_t (*)(const LdsArgs&, hipStream_t);
using MultiFn = hipError_t (*)(const MultiArgs&, int32_t, hipStream_t);
const OneFn kOne[][2] = {SDD_LDS_SHAPES(SDD_ONE_PTR)};
const MultiFn kMulti[][2] = {SDD_LDS_SHAPES(SDD_MULTI_PTR)};
}  // namespace

hipError_t launch_dedisperse_lds(const LdsArgs& a, int shape, hipStream_t s) {
  if (shape < 0 || shape >= kNumLdsShapes || a.es < 1 || a.es > 2) return hipErrorInvalidValue;
  return kOne[shape][a.es - 1](a, s);
}

hipError_t launch_dedisperse_lds_multi(const MultiArgs& m, int32_t max_win, int shape,
                                       hipStream_t s) {
  if (shape < 0 || shape >= kNumLdsShapes || m.njobs < 1) return hipErrorInvalidValue;
  const int es = m.jobs[0].es;
  for (int j = 1; j < m.njobs; ++j)
    if (m.jobs[j].es != es) return hipErrorInvalidValue;
  if (es < 1 || es > 2) return hipErrorInvalidValue;
  return kMulti[shape][es - 1](m, max_win, s);
}

}  // namespace sdd
