// Matrix-core form of the LDS-tiled dedispersion (Section 3.2: every trial
// DM sums all channels along its delay curve, plane[i][j] = sum_c
// x[c][j + delay[c][i]]), for uint8 channel rows. Included by
// k_dedisp_lds.hip inside its anonymous namespace.
//
// The channel sum with its per-channel shift is written as a product of a
// 0/1 selection matrix and the staged input bytes, which one
// v_mfma_i32_16x16x64_i8 evaluates for two channels at once:
//   C[j][n] += sum_{q<2} sum_{b<32} S_q[j][b] * X_q[b][n],
//   X_q[b][n] = window byte P_q + 16 n + b of channel q (as x - 128),
//   S_q[j][b] = 1 when b == j + r_q,
// where p_q = P_q + r_q (P_q a multiple of 16, r_q < 16) is the trial's
// offset into the channel's staged window. Column n of C is 16 consecutive
// samples, so one product adds two channels into 256 samples of one trial.
// The operands in lane order: lane l = n + 16 g (n < 16, g < 4) holds 16
// bytes of K slots 16 g .. 16 g + 15, i.e. bytes 16 (g & 1) .. + 15 of the
// 32-byte segment of channel q = g >> 1; the selection operand of lane l is
// row n of S_q over the same slots, a one-hot 16-byte word read from a
// 1 KiB table in LDS. Sums stay in int32 accumulators for the whole channel
// loop (no 16-bit flushes); each staged byte is x ^ 0x80 (x - 128 as int8),
// so the stored value is C + 128 * (channels summed). Padding channels past
// nchan and bytes past a row's end are staged as 0x80 (value 0).
//
// Per wavefront: D trials x MT blocks of 256 samples; per (channel pair,
// trial) one table read, MT 16-byte data reads and MT products. Staging
// keeps one copy per channel (16-byte aligned windows), double-buffered by
// stage as in the vector form. AHEAD > 0 pins the order of a stage's reads
// and products with scheduling groups so that AHEAD reads are in flight
// when a product issues (left alone, the compiler issues each read one or
// two ahead of its product, too few to cover the LDS latency at 4
// wavefronts per SIMD).

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

template <int D, int MT, int WD, int WT, int CS, int NLD, bool INTERIOR, bool SHARE, int AHEAD>
__device__ __forceinline__ void mf_tile_impl(const LdsArgs& a, int32_t dtile, int32_t ttile,
                                             uint8_t* __restrict__ lds) {
  constexpr int NT = 64 * WD * WT;
  constexpr int DT = D * WD;
  constexpr int TW = 256 * MT;  // samples per time group of waves
  constexpr int TT = TW * WT;
  constexpr int NE = (CS / 2) * D;  // (channel pair, trial) entries per wavefront and stage
  static_assert(CS % 2 == 0, "channels are taken in pairs");
  static_assert(NE <= 64, "one entry per lane");
  // The last stage is padded with empty channels up to CS, and their delay
  // rows are read unmasked: the table's zero rows (to a multiple of
  // kDelayRowPad) must cover every padded stage, so CS must divide it.
  static_assert(kDelayRowPad % CS == 0, "stage must divide the delay-table padding");
  static_assert(CS * (TT + 32) <= 16 * NLD * NT, "staging too small for the tile");
  const int32_t i0 = dtile * DT;
  const int64_t t0 = (int64_t)ttile * TT;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wd = wave % WD, wt = wave / WD;
  const int32_t ndm = a.ndm, nchan = a.nchan;
  const int32_t win = a.win;      // bytes per channel window, multiple of 16
  const int32_t buf = CS * win;   // one stage buffer
  const int32_t wq = win >> 4;
  const int64_t pitch = a.x_pitch;
  const int64_t row_bytes = a.x_len;
  const int32_t tab = 2 * buf;    // selection table: [h < 2][t < 32] x 16 bytes

  // table entry (h, t): byte k is 1 when 16 h + k == t
  if (tid < 64) {
    const int h = tid >> 5, t = tid & 31, k = t - 16 * h;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (k >= 0 && k < 16 && (k >> 2) == e) w[e] = 1u << (8 * (k & 3));
    *reinterpret_cast<u32x4*>(lds + tab + 512 * h + 16 * t) = u32x4{w[0], w[1], w[2], w[3]};
  }

  i32x4 acc[D][MT];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[d][m] = i32x4{0, 0, 0, 0};

  // ---- staging: global -> registers -> LDS (x ^ 0x80) ----
  int32_t ecs[NLD];    // slot, CS for an unused element
  uint32_t eoff[NLD];  // cs * pitch + 16 q
  int32_t eq16[NLD];   // 16 q
  uint32_t ebase[NLD]; // (cs * ndm + i0) * 4
  int32_t elds[NLD];   // cs * win + 16 q
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int32_t e = tid + k * NT;
    const int32_t cs = e / wq;
    const int32_t q = e - cs * wq;
    ecs[k] = cs < CS ? cs : CS;
    const int32_t csv = cs < CS ? cs : 0;
    eoff[k] = (uint32_t)(csv * pitch) + 16u * (uint32_t)q;
    eq16[k] = 16 * q;
    ebase[k] = 4u * (uint32_t)(csv * ndm + i0);
    elds[k] = csv * win + 16 * q;
  }
  const uint8_t* __restrict__ xs = a.x + t0;
  const uint8_t* __restrict__ ds = reinterpret_cast<const uint8_t*>(a.delays);
  const int64_t stage_drow = 4 * (int64_t)CS * ndm;
  u32x4 st[NLD];
  bool live[NLD];  // false: a padding channel (staged as zeros)
  auto load_bases = [&](int32_t s, int32_t (&dst)[NLD]) {
    const uint8_t* row = ds + (int64_t)s * stage_drow;
#pragma unroll
    for (int k = 0; k < NLD; ++k) dst[k] = *reinterpret_cast<const int32_t*>(row + ebase[k]);
  };
  // The loads stay in flight until store_stage at the end of the stage: no
  // use of st before then. A padding channel (past nchan, only in the last
  // stage) loads row 0 instead and is staged as zeros.
  auto load_data = [&](int32_t s, const int32_t (&bases)[NLD]) {
    const uint8_t* row = xs + (int64_t)s * CS * pitch;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const bool real = s * CS + ecs[k] < nchan;
      const uint8_t* src = row + eoff[k] + (uint32_t)(bases[k] & ~15);
      if constexpr (INTERIOR) {
        st[k] = *reinterpret_cast<const u32x4*>(real ? src : xs + eq16[k]);
        live[k] = real;
      } else {
        live[k] = true;
        u32x4 v = u32x4{0u, 0u, 0u, 0u};
        if (real) {
          const int64_t g = t0 + (bases[k] & ~15) + eq16[k];  // byte g of the row; zero past its end
          if (a.aligned && g + 16 <= row_bytes) {
            v = *reinterpret_cast<const u32x4*>(src);
          } else {
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            for (int bb = 0; bb < 16; ++bb)
              if (g + bb < row_bytes) w[bb >> 2] |= (uint32_t)src[bb] << (8 * (bb & 3));
            v = u32x4{w[0], w[1], w[2], w[3]};
          }
        }
        st[k] = v;
      }
    }
  };
  auto store_stage = [&](int32_t s) {
    uint8_t* base = lds + (s & 1) * buf;
#pragma unroll
    for (int k = 0; k < NLD; ++k)
      if (ecs[k] < CS)
        *reinterpret_cast<u32x4*>(base + elds[k]) =
            (live[k] ? st[k] : u32x4{0u, 0u, 0u, 0u}) ^ 0x80808080u;
  };

  // ---- read positions: lane k < NE holds entry k = pair * D + d ----
  // PP: LDS offsets / 16 (stage buffer, slot, 16-aligned window offset) of
  // the pair's two channels in the low and high halves; RR: r of each.
  uint32_t dlA, dlA0, dlB, dlB0;
  {
    const int32_t k = lane < NE ? lane : 0;
    const int32_t p = k / D, d = k - p * D;
    const int32_t i = i0 + wd * D + d;
    const int32_t ic = i < ndm ? i : ndm - 1;
    dlA = 4u * (uint32_t)(2 * p * ndm + ic);
    dlA0 = 4u * (uint32_t)(2 * p * ndm + i0);
    dlB = dlA + 4u * (uint32_t)ndm;
    dlB0 = dlA0 + 4u * (uint32_t)ndm;
  }
  const int32_t pA = 2 * ((lane < NE ? lane : 0) / D);  // first channel of the lane's pair
  int32_t wA, wA0, wB, wB0;
  auto load_words = [&](int32_t s) {
    const uint8_t* row = ds + (int64_t)s * stage_drow;
    wA = *reinterpret_cast<const int32_t*>(row + dlA);
    wA0 = *reinterpret_cast<const int32_t*>(row + dlA0);
    wB = *reinterpret_cast<const int32_t*>(row + dlB);
    wB0 = *reinterpret_cast<const int32_t*>(row + dlB0);
  };
  auto pack_words = [&](int32_t s, uint32_t& pp, uint32_t& rr) {
    const int32_t oA = wA - (wA0 & ~15), oB = wB - (wB0 & ~15);
    const int32_t bo = (s & 1) * buf + pA * win;
    // offsets in 16-byte units (every one is 16-aligned): 16 bits hold 1 MiB
    pp = (uint32_t)((bo + (oA & ~15)) >> 4) | ((uint32_t)((bo + win + (oB & ~15)) >> 4) << 16);
    rr = (uint32_t)(oA & 15) | ((uint32_t)(oB & 15) << 16);
  };

  // lane constants: column n, K group g = 2 q + h
  const int n = lane & 15, g4 = lane >> 4;
  const uint32_t lane_sh = 16u * (uint32_t)(g4 >> 1);
  const uint32_t lane_b = 16u * (uint32_t)(n + (g4 & 1)) + (uint32_t)(TW * wt);
  const uint32_t lane_t = (uint32_t)tab + 512u * (uint32_t)(g4 & 1) + 16u * (uint32_t)n;

  struct Grp {
    i32x4 sel;
    i32x4 x[MT];
  };
  auto fetch = [&](uint32_t ppv, uint32_t rrv, int e, Grp& r) {
    const uint32_t pp = (uint32_t)__builtin_amdgcn_readlane((int)ppv, e);
    const uint32_t rr = (uint32_t)__builtin_amdgcn_readlane((int)rrv, e);
    const uint32_t ab = (__builtin_amdgcn_ubfe(pp, lane_sh, 16) << 4) + lane_b;
    const uint32_t at = (__builtin_amdgcn_ubfe(rr, lane_sh, 16) << 4) + lane_t;
    r.sel = *reinterpret_cast<const i32x4*>(lds + at);
#pragma unroll
    for (int m = 0; m < MT; ++m) r.x[m] = *reinterpret_cast<const i32x4*>(lds + ab + 256 * m);
  };
  auto consume = [&](int e, const Grp& r) {
    const int d = e % D;
#pragma unroll
    for (int m = 0; m < MT; ++m)
      acc[d][m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(r.sel, r.x[m], acc[d][m], 0, 0, 0);
  };

  const int32_t nstages = (nchan + CS - 1) / CS;  // the last one padded with empty channels
  uint32_t ppn = 0, rrn = 0;
  int32_t bnext[NLD];
  {
    int32_t b0[NLD];
    load_bases(0, b0);
    load_words(0);
    load_data(0, b0);
    if (nstages > 1) load_bases(1, bnext);
    pack_words(0, ppn, rrn);
    store_stage(0);
  }
  __syncthreads();
  for (int32_t s = 0; s < nstages; ++s) {
    const uint32_t ppc = ppn, rrc = rrn;
    if (s + 1 < nstages) {
      load_data(s + 1, bnext);
      load_words(s + 1);
      if (s + 2 < nstages) load_bases(s + 2, bnext);
    }
    if constexpr (SHARE) {
      // Trials of one wavefront are neighbours: when a channel pair's two
      // windows start in the same 16-byte words for trial d as for trial
      // d - 1 (equal packed offsets), the data operands are the same and
      // only the selection differs, so the data reads are skipped.
      constexpr int NP = CS / 2;
      struct Pair {
        uint32_t pp[D];
        i32x4 sel[D];
        i32x4 x[MT];
      };
      auto fetch_pair = [&](int p, Pair& r) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          r.pp[d] = (uint32_t)__builtin_amdgcn_readlane((int)ppc, p * D + d);
          const uint32_t rr = (uint32_t)__builtin_amdgcn_readlane((int)rrc, p * D + d);
          const uint32_t at = (__builtin_amdgcn_ubfe(rr, lane_sh, 16) << 4) + lane_t;
          r.sel[d] = *reinterpret_cast<const i32x4*>(lds + at);
        }
        const uint32_t ab = (__builtin_amdgcn_ubfe(r.pp[0], lane_sh, 16) << 4) + lane_b;
#pragma unroll
        for (int m = 0; m < MT; ++m) r.x[m] = *reinterpret_cast<const i32x4*>(lds + ab + 256 * m);
      };
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        Pair c;
        fetch_pair(p, c);
#pragma unroll
        for (int m = 0; m < MT; ++m)
          acc[0][m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(c.sel[0], c.x[m], acc[0][m], 0, 0, 0);
#pragma unroll
        for (int d = 1; d < D; ++d) {
          if (c.pp[d] == c.pp[0]) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
              acc[d][m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(c.sel[d], c.x[m], acc[d][m], 0, 0, 0);
          } else {
            const uint32_t ab = (__builtin_amdgcn_ubfe(c.pp[d], lane_sh, 16) << 4) + lane_b;
            i32x4 y[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) y[m] = *reinterpret_cast<const i32x4*>(lds + ab + 256 * m);
#pragma unroll
            for (int m = 0; m < MT; ++m)
              acc[d][m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(c.sel[d], y[m], acc[d][m], 0, 0, 0);
          }
        }
      }
    } else {
      Grp gr[2];
      fetch(ppc, rrc, 0, gr[0]);
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        if (e + 1 < NE) fetch(ppc, rrc, e + 1, gr[(e + 1) & 1]);
        consume(e, gr[e & 1]);
      }
      if constexpr (AHEAD > 0) {
        // The stage's order: the first group's selection read and AHEAD data
        // reads, then one read after each product, two where the next group's
        // selection read falls, so every product finds AHEAD reads issued
        // past its own (masks: 0x100 LDS reads, 0x008 matrix products).
        static_assert(AHEAD < MT, "look-ahead within a group");
        __builtin_amdgcn_sched_group_barrier(0x100, 1 + AHEAD, 0);
#pragma unroll
        for (int t = 0; t < NE * MT; ++t) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          if ((t % MT) == MT - 1 - AHEAD)
            __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
          else
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
      }
    }
    if (s + 1 < nstages) {
      store_stage(s + 1);
      pack_words(s + 1, ppn, rrn);
    }
    __syncthreads();
  }

  // ---- store the tile: lane l holds samples 16 n + 4 g .. + 3 of each block ----
  const int32_t corr = 128 * CS * nstages;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int32_t i = i0 + wd * D + d;
    if (i >= ndm) break;
    uint32_t* row = a.plane + (int64_t)i * a.plane_pitch;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int64_t j = t0 + TW * wt + 256 * m + 16 * n + 4 * g4;
      const uint32_t v0 = (uint32_t)(acc[d][m][0] + corr), v1 = (uint32_t)(acc[d][m][1] + corr);
      const uint32_t v2 = (uint32_t)(acc[d][m][2] + corr), v3 = (uint32_t)(acc[d][m][3] + corr);
      if (j + 4 <= a.cols) {
        *reinterpret_cast<uint4*>(row + j) = make_uint4(v0, v1, v2, v3);
      } else {
        if (j < a.cols) row[j] = v0;
        if (j + 1 < a.cols) row[j + 1] = v1;
        if (j + 2 < a.cols) row[j + 2] = v2;
      }
    }
  }
}
