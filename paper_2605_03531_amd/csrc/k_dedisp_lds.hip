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
// Workgroups are ordered time-tile-major and each XCD takes a contiguous run of
// tiles, so the concurrently running tiles of one XCD are neighbouring DM
// tiles of the same time tile: for every channel their windows overlap by at
// least the tile length, and the input one tile loads is mostly already in
// that XCD's L2 (a DM-tile-major order re-reads the whole input from HBM once
// per DM tile).
#include "k_dedisp_lds.h"

namespace sdd {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One DT x TT tile of one job. Every thread of the workgroup calls it; it
// returns after a barrier, so the caller may reuse the LDS at once.
// ES = input element bytes: 1 (uint8 rows) or 2 (uint16 rows of a decimated
// range). A lane always owns 8 bytes of a 512-byte chunk: 8 uint8 samples
// (four 16-bit pairs after widening) or 4 uint16 samples (two pairs as read).
// INTERIOR: every staging load of the tile lies inside the rows and the rows
// are 16-byte aligned, so the loads need no per-element checks.
// Flag 8 (uint16 rows only): each window is kept as four copies shifted by 0,
// 2, 4 and 6 bytes, so every sample position a lane reads starts an aligned
// 8-byte word of one of them: a channel costs one conflict-free 64-bit read
// per 4 samples, and a channel pair one v_add3 per packed word, where two
// copies (0 and 4 bytes) need a 2-way bank-conflicted 32-bit read and two
// v_perm alignments per channel as well.
template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES, bool INTERIOR>
__device__ __forceinline__ void dd_tile_impl(const LdsArgs& a, int32_t dtile, int32_t ttile,
                                             uint8_t* __restrict__ lds) {
  constexpr int NT = 64 * WD * WT;
  constexpr int DT = D * WD;
  constexpr int SPL = 8 / ES;       // samples per lane per chunk
  constexpr int CH = 64 * SPL;      // samples per 512-byte chunk
  constexpr int NPK = SPL / 2;      // packed 16-bit pairs per lane per chunk
  constexpr int TW = CH * M;        // samples per time group of waves
  constexpr int TT = TW * WT;
  constexpr bool WIDE = (F & 2) != 0;  // third word through a 64-bit read
  constexpr bool FOUR = (F & 8) != 0;  // four shifted copies per window
  constexpr int NCOPY = FOUR ? 4 : 2;
  static_assert(!FOUR || ES == 2, "four-copy windows hold uint16 rows");
  static_assert(!FOUR || !WIDE, "four-copy windows read whole words");
  constexpr int NDV = (CS * D + 63) / 64;  // VGPRs holding one stage's read positions
  static_assert(CS % 2 == 0, "channels are added in pairs");
  // the staging must hold a stage's windows at zero delay span at least
  static_assert(CS * (ES * TT + 32 * ES) <= 16 * NLD * NT, "staging too small for the tile");
  const int32_t i0 = dtile * DT;
  const int64_t t0 = (int64_t)ttile * TT;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wd = wave % WD, wt = wave / WD;
  const int32_t ndm = a.ndm, nchan = a.nchan;
  const int32_t win = a.win;            // bytes per copy, multiple of 16
  const int32_t slot = NCOPY * win;     // the copies of one window
  const int32_t buf = CS * slot;
  const int32_t wq = win >> 4;          // 16-byte elements per window
  const int64_t pitch_bytes = (int64_t)ES * a.x_pitch;
  const int64_t row_bytes = (int64_t)ES * a.x_len;

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
  // Thread element k covers 16 bytes (q) of the window of slot ecs[k]. Its
  // loads address (uniform stage base) + (32-bit per-lane offset); the
  // window starts at sample t0 + (d(c, i0) & ~15), with d(c, i0) loaded two
  // stages ahead by the element itself.
  int32_t ecs[NLD];     // slot, CS for an unused element
  uint32_t eoff[NLD];   // cs * pitch + 16 q (bytes from the stage's row base)
  int32_t eq16[NLD];    // 16 q
  uint32_t ebase[NLD];  // (cs * ndm + i0) * 4 (bytes from the stage's first delay row)
  int32_t elds[NLD];    // cs * slot + 16 q
#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int32_t e = tid + k * NT;
    const int32_t cs = e / wq;
    const int32_t q = e - cs * wq;
    ecs[k] = cs < CS ? cs : CS;
    // an unused element loads (and never stores) a valid window of slot 0
    const int32_t csv = cs < CS ? cs : 0;
    eoff[k] = (uint32_t)(csv * pitch_bytes) + 16u * (uint32_t)q;
    eq16[k] = 16 * q;
    ebase[k] = 4u * (uint32_t)(csv * ndm + i0);
    elds[k] = csv * slot + 16 * q;
  }
  const uint8_t* __restrict__ xs = a.x + ES * t0;  // stage 0 row base (uniform)
  // stage 0 delay row base (uniform); the table has zero rows up to a
  // multiple of kDelayRowPad channels, so every stage reads it unmasked
  const uint8_t* __restrict__ ds = reinterpret_cast<const uint8_t*>(a.delays);
  const int64_t stage_drow = 4 * (int64_t)CS * ndm;  // delay-table bytes per stage
  static_assert(CS <= kDelayRowPad, "stage wider than the delay-table padding");

  // copy 0 and copy 1 of each element as loaded (copy 1 is the same window
  // 4 bytes on: a second 16-byte load from L1 costs no register moves); with
  // four copies, bytes 0-15 and 8-23 of the element, from which the copies
  // are formed at the store
  u32x4 st0[NLD], st1[NLD];
  constexpr int LB = FOUR ? 24 : 20;  // bytes of the row an element loads
  // d(c, i0) of each element's channel at a stage
  auto load_bases = [&](int32_t s, int32_t (&dst)[NLD]) {
    const uint8_t* row = ds + (int64_t)s * stage_drow;
#pragma unroll
    for (int k = 0; k < NLD; ++k) dst[k] = *reinterpret_cast<const int32_t*>(row + ebase[k]);
  };
  // Stages cover whole groups of CS channels; the nchan % CS channels left
  // over are added after the loop.
  auto load_data = [&](int32_t s, const int32_t (&bases)[NLD]) {
    const uint8_t* row = xs + (int64_t)s * CS * pitch_bytes;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const uint32_t off = eoff[k] + (uint32_t)(ES * (bases[k] & ~15));
      const uint8_t* src = row + off;
      if constexpr (INTERIOR) {
        st0[k] = *reinterpret_cast<const u32x4*>(src);
        st1[k] = *reinterpret_cast<const u32x4*>(src + (LB == 24 ? 8 : 4));
      } else {
        // byte g of the row; zero past its end
        const int64_t g = ES * (t0 + (bases[k] & ~15)) + eq16[k];
        uint32_t w[LB / 4] = {};
        if (a.aligned && g + LB <= row_bytes) {
          const uint4 t = *reinterpret_cast<const uint4*>(src);
          w[0] = t.x; w[1] = t.y; w[2] = t.z; w[3] = t.w;
          w[4] = *reinterpret_cast<const uint32_t*>(src + 16);
          if constexpr (LB == 24) w[5] = *reinterpret_cast<const uint32_t*>(src + 20);
        } else {
          for (int bb = 0; bb < LB; ++bb)
            if (g + bb < row_bytes) w[bb >> 2] |= (uint32_t)src[bb] << (8 * (bb & 3));
        }
        st0[k] = u32x4{w[0], w[1], w[2], w[3]};
        if constexpr (LB == 24)
          st1[k] = u32x4{w[2], w[3], w[4], w[5]};
        else
          st1[k] = u32x4{w[1], w[2], w[3], w[4]};
      }
    }
  };
  auto store_stage = [&](int32_t s) {
    uint8_t* base = lds + (s & 1) * buf;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      if (ecs[k] < CS) {
        uint8_t* c0 = base + elds[k];
        if constexpr (FOUR) {
          // copy n byte j = window byte j + 2n, from words w0-w5 of the element
          const uint32_t w0 = st0[k].x, w1 = st0[k].y, w2 = st0[k].z, w3 = st0[k].w;
          const uint32_t w4 = st1[k].z, w5 = st1[k].w;
          // bytes 2-5 of the pair (lo, hi)
          auto mid = [](uint32_t lo, uint32_t hi) { return (lo >> 16) | (hi << 16); };
          const uint32_t h1 = mid(w1, w2), h2 = mid(w2, w3), h3 = mid(w3, w4);
          *reinterpret_cast<u32x4*>(c0) = st0[k];
          *reinterpret_cast<u32x4*>(c0 + win) = u32x4{mid(w0, w1), h1, h2, h3};
          *reinterpret_cast<u32x4*>(c0 + 2 * win) = u32x4{w1, w2, w3, w4};
          *reinterpret_cast<u32x4*>(c0 + 3 * win) = u32x4{h1, h2, h3, mid(w4, w5)};
        } else {
          // copy 0 as loaded; copy 1 byte j = window byte j + 4
          *reinterpret_cast<u32x4*>(c0) = st0[k];
          *reinterpret_cast<u32x4*>(c0 + win) = st1[k];
        }
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

  // Read positions of a stage: lane k < CS*D holds entry k = slot*D + d,
  // trial d of this wavefront in that slot's channel, packed as bits 0-19 the
  // LDS byte offset of its 8-byte word from the stage buffer (the slot's
  // offset, plus the copy that starts the word at the position: copy 1 when
  // the offset within the word is >= 4, or copy (offset within the word) / 2
  // of four; at most CS * NCOPY * win < 160 KiB) and bits 20-21 the remaining
  // byte shift (always 0 with four copies).
  // They are computed here across the lanes, once per stage, so the compute
  // loop needs one v_readlane and a few scalar operations per channel and
  // trial, and no scalar-memory waits that would also drain its LDS reads.
  // A channel past nchan gets offset 0 into its all-zero window.
  uint32_t dl_off[NDV], dl_off0[NDV];  // bytes from the stage's first delay row
  int32_t sl_off[NDV];                  // the entry's slot offset in the stage buffer
#pragma unroll
  for (int v = 0; v < NDV; ++v) {
    const int32_t k = 64 * v + lane;
    const int32_t cs = k / D, d = k - cs * D;
    const int32_t i = i0 + wd * D + d;
    const int32_t csv = k < CS * D ? cs : 0;
    dl_off[v] = 4u * (uint32_t)(csv * ndm + (i < ndm ? i : ndm - 1));
    dl_off0[v] = 4u * (uint32_t)(csv * ndm + i0);
    sl_off[v] = csv * slot;
  }
  int32_t rdv[NDV], rd0[NDV];
  auto load_words = [&](int32_t s) {
    const uint8_t* row = ds + (int64_t)s * stage_drow;
#pragma unroll
    for (int v = 0; v < NDV; ++v) {
      rdv[v] = *reinterpret_cast<const int32_t*>(row + dl_off[v]);
      rd0[v] = *reinterpret_cast<const int32_t*>(row + dl_off0[v]);
    }
  };
  auto pack_words = [&](int32_t (&out)[NDV]) {
#pragma unroll
    for (int v = 0; v < NDV; ++v) {
      const int32_t o = ES * (rdv[v] - (rd0[v] & ~15));
      if constexpr (FOUR) {
        out[v] = sl_off[v] + (o & ~7) + ((o >> 1) & 3) * win;
      } else {
        const int32_t ad = (o & ~7) + ((o & 4) ? win : 0);
        out[v] = (sl_off[v] + ad) | ((o & 3) << 20);
      }
    }
  };

  // entry k of the current stage, as a wave-uniform scalar
#define SDD_WORD(k) __builtin_amdgcn_readlane(dcur[(k) / 64], (k) % 64)

  // One group: channels cc, cc+1 of a stage, trial d of the wavefront. Its
  // reads (12 bytes per chunk per channel) and v_perm selectors.
  constexpr int NG = (CS / 2) * D;
  struct Grp {
    uint2 a01[M], b01[M];
    uint32_t a2[M], b2[M];
    uint32_t sA0, sB0;
  };
  auto fetch = [&](const uint8_t* bufp, const int32_t (&dcur)[NDV], int g, Grp& r) {
    const int cc = 2 * (g / D), d = g % D;
    const uint32_t wA = (uint32_t)SDD_WORD(cc * D + d);
    const uint32_t wB = (uint32_t)SDD_WORD((cc + 1) * D + d);
    const int32_t adA = (int32_t)(wA & 0xfffffu);
    const int32_t adB = (int32_t)(wB & 0xfffffu);
    const uint32_t rA = wA >> 20, rB = wB >> 20;
    // v_perm selectors: bytes r, r+1 (and r+2, r+3) into 16-bit fields for
    // uint8 input; bytes r..r+3 in order for uint16 input
    r.sA0 = ES == 1 ? 0x0c010c00u + rA * 0x00010001u : 0x03020100u + rA * 0x01010101u;
    r.sB0 = ES == 1 ? 0x0c010c00u + rB * 0x00010001u : 0x03020100u + rB * 0x01010101u;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      int32_t oA = adA + 512 * m, oB = adB + 512 * m;
      if constexpr (FOUR) {
        // A register address per chunk: with one base and offsets 512 apart
        // the compiler fuses the chunks' reads into one ds_read2st64_b64,
        // which moves half the bytes per clock of two ds_read_b64.
        if (m > 0) asm volatile("" : "+s"(oA), "+s"(oB));
      }
      const uint8_t* pA = bufp + oA;
      const uint8_t* pB = bufp + oB;
      r.a01[m] = *reinterpret_cast<const uint2*>(pA);
      r.b01[m] = *reinterpret_cast<const uint2*>(pB);
      if constexpr (FOUR) {
        // the word holds the lane's 4 samples in place
        r.a2[m] = r.b2[m] = 0u;
      } else if constexpr (WIDE) {
        const uint2 a23 = *reinterpret_cast<const uint2*>(pA + 8);
        const uint2 b23 = *reinterpret_cast<const uint2*>(pB + 8);
        // keep the full 64-bit reads (conflict-free at an 8-byte lane stride)
        asm volatile("" ::"v"(a23.y), "v"(b23.y));
        r.a2[m] = a23.x;
        r.b2[m] = b23.x;
      } else {
        r.a2[m] = *reinterpret_cast<const uint32_t*>(pA + 8);
        r.b2[m] = *reinterpret_cast<const uint32_t*>(pB + 8);
      }
    }
  };
  auto consume = [&](int g, const Grp& r) {
    const int d = g % D;
    const uint32_t sA0 = r.sA0, sB0 = r.sB0;
    const uint32_t sA2 = sA0 + 0x00020002u;
    const uint32_t sB2 = sB0 + 0x00020002u;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const uint2 a01 = r.a01[m], b01 = r.b01[m];
      const uint32_t a2 = r.a2[m], b2 = r.b2[m];
      if constexpr (FOUR) {
        acc[d][m][0] += a01.x + b01.x;
        acc[d][m][1] += a01.y + b01.y;
      } else if constexpr (ES == 1) {
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
      // add this group into the accumulators now: left to itself the
      // compiler keeps a group's widened words live to sum them with the
      // next group's, which costs the registers the pipelining needs
#pragma unroll
      for (int k = 0; k < NPK; ++k) asm volatile("" : "+v"(acc[d][m][k]));
    }
  };

  const int32_t nstages = nchan / CS;  // whole stages
  const int32_t lane_off = 8 * lane + ES * TW * wt;  // bytes
  const int32_t fstages = (ES == 1 ? 256 : a.flush) / CS;
  int32_t fl = fstages;
  int32_t dnext[NDV];
  int32_t bnext[NLD];
  if (nstages > 0) {
    int32_t b0[NLD];
    load_bases(0, b0);
    load_words(0);
    load_data(0, b0);
    if (nstages > 1) load_bases(1, bnext);
    pack_words(dnext);
    store_stage(0);
  }
  __syncthreads();
  for (int32_t s = 0; s < nstages; ++s) {
    int32_t dcur[NDV];
#pragma unroll
    for (int v = 0; v < NDV; ++v) dcur[v] = dnext[v];
    if (s + 1 < nstages) {
      // stage s+1: data (its bases arrived a stage ago) and read positions;
      // stage s+2: window bases
      load_data(s + 1, bnext);
      load_words(s + 1);
      if (s + 2 < nstages) load_bases(s + 2, bnext);
    }
    const uint8_t* bufp = lds + (s & 1) * buf + lane_off;
    // The stage's (channel pair, trial) groups are software-pipelined: the LDS
    // reads of group g+1 are issued before group g is widened and added, so
    // each wavefront has a group's reads in flight while it computes.
    Grp gr[2];
    fetch(bufp, dcur, 0, gr[0]);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      if (g + 1 < NG) fetch(bufp, dcur, g + 1, gr[(g + 1) & 1]);
      consume(g, gr[g & 1]);
    }
    if (--fl == 0 || s + 1 == nstages) {
      flush();
      fl = fstages;
    }
    if (s + 1 < nstages) {
      store_stage(s + 1);
      pack_words(dnext);
    }
    __syncthreads();
  }

#undef SDD_WORD

  // ---- the nchan % CS channels past the last whole stage, from global ----
  for (int32_t c = nstages * CS; c < nchan; ++c) {
    const uint8_t* xrow = a.x + (int64_t)c * pitch_bytes;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int32_t i = i0 + wd * D + d;
      const int32_t dl = a.delays[(int64_t)c * ndm + (i < ndm ? i : ndm - 1)];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int64_t j = t0 + TW * wt + CH * m + SPL * lane + dl;
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
          if (j + k < a.x_len)
            wide[d][m][k] += ES == 1 ? (uint32_t)xrow[j + k]
                                     : (uint32_t)reinterpret_cast<const uint16_t*>(xrow)[j + k];
        }
      }
    }
  }

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

#include "k_dedisp_mfma.h"

// Reads the matrix-core loop keeps in flight ahead of its products (0: the
// compiler's order), measured per shape on the full-band chunk: the
// one-trial, 2048-sample, 16-channel-stage shape 51.9 ms with 4 against 55.6
// ms with 0 (3: 52.5, 5: 52.1), and its persistent form over 32 beams 1.070 s
// with 4 against 1.074 (3), 1.103 (2) and 1.128 s (0), though it keeps 64
// bytes per lane in scratch at 4; the two-trial shapes spill from 4 on and
// were no faster with 2 or 3, so they keep 0.
template <int D, int M, int CS>
constexpr int kMfAhead = (D == 1 && M == 4 && CS == 16) ? 4 : 0;

// Shapes with flag 4 take the matrix-core form (uint8 rows only; its
// launchers refuse uint16 jobs), with M 512-sample chunks = 2 M products of
// 256 samples per trial and wavefront; shapes with flag 8 take uint16 rows
// only.
template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
__device__ __forceinline__ void dd_tile(const LdsArgs& a, int32_t dtile, int32_t ttile,
                                        uint8_t* __restrict__ lds) {
  if constexpr ((F & 8) != 0 && ES != 2) {
    // four-copy shapes take uint16 rows only; their launchers refuse the rest
  } else if constexpr ((F & 4) != 0) {
    constexpr bool SHARE = (F & 16) != 0;
    constexpr int AH = kMfAhead<D, M, CS>;
    if (ttile < a.n_tt_interior)
      mf_tile_impl<D, 2 * M, WD, WT, CS, NLD, true, SHARE, AH>(a, dtile, ttile, lds);
    else
      mf_tile_impl<D, 2 * M, WD, WT, CS, NLD, false, SHARE, AH>(a, dtile, ttile, lds);
  } else {
    if (ttile < a.n_tt_interior)
      dd_tile_impl<D, M, WD, WT, CS, NLD, F, ES, true>(a, dtile, ttile, lds);
    else
      dd_tile_impl<D, M, WD, WT, CS, NLD, F, ES, false>(a, dtile, ttile, lds);
  }
}

// Matrix-core shapes are held to 128 VGPRs (4 wavefronts per SIMD, two
// 512-thread workgroups per CU): left free, the persistent form's extra
// state took its 16-channel shape to 138 (one workgroup per CU, 25%
// slower); held, it keeps a few values in scratch and runs as fast as the
// grid form.
template <int F>
constexpr int kWavesPerSimd = (F & 4) != 0 ? 4 : 1;

// Dynamic LDS of one workgroup: two stage buffers of CS windows, with two
// copies per window in the vector form (four with flag 8), one plus the 1 KiB
// selection table in the matrix-core form.
template <int CS, int F>
constexpr size_t tile_lds_bytes(int32_t win) {
  return (F & 4) != 0 ? (size_t)2 * CS * win + 1024
                      : (size_t)2 * CS * ((F & 8) != 0 ? 4 : 2) * win;
}
// The kinds of rows a shape's form takes: the matrix-core form uint8 only,
// the four-copy vector form uint16 only.
template <int F, int ES>
constexpr bool takes_rows() {
  return (F & 4) != 0 ? ES == 1 : (F & 8) != 0 ? ES == 2 : true;
}

// Grid form: one workgroup per tile of one job, ordered time-tile-major with a
// contiguous run of tiles per XCD (workgroups go to the 8 XCDs round-robin).
template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
__global__ __launch_bounds__(64 * WD * WT, kWavesPerSimd<F>) void k_dedisp_lds(LdsArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int32_t nblk = a.n_dtiles * a.n_ttiles;
  const int32_t b = blockIdx.x;
  const int32_t full = nblk & ~7;
  const int32_t L = b < full ? (b & 7) * (full >> 3) + (b >> 3) : b;
  const int32_t ttile = L / a.n_dtiles;
  dd_tile<D, M, WD, WT, CS, NLD, F, ES>(a, L - ttile * a.n_dtiles, ttile, lds);
}

// Persistent form for a batch of jobs (beams x DM ranges with the same tile
// shape): the global tile list (job by job, time-tile-major inside a job) is
// cut into 8 contiguous parts, one per XCD. The workgroups of an XCD take the
// tiles of its part in order from a counter of that XCD, each workgroup its
// next tile when it finishes one (as the hardware hands out the workgroups of
// a grid), so the tiles running together on an XCD are the latest few dozen
// of its part: neighbours that share input in its L2. (A fixed assignment,
// tile r * n + k to workgroup k in round r, lets the workgroups drift apart
// by many rounds over a long batch and loses that sharing.)
template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
__global__ __launch_bounds__(64 * WD * WT, kWavesPerSimd<F>) void k_dedisp_lds_multi(MultiArgs m) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  __shared__ int32_t ticket;
  const int32_t total = m.tile_base[m.njobs];
  const int xcd = blockIdx.x & 7;                  // workgroups go to XCDs round-robin
  const int32_t lo = (int32_t)(((int64_t)total * xcd) >> 3);
  const int32_t hi = (int32_t)(((int64_t)total * (xcd + 1)) >> 3);
  int j = 0;
  for (;;) {
    // every thread reads the ticket before the tile's first barrier, so the
    // next write (after the tile's last barrier) cannot overtake a read
    if (threadIdx.x == 0) ticket = (int32_t)atomicAdd(m.tickets + xcd, 1u);
    __syncthreads();
    const int32_t t = lo + ticket;
    if (t >= hi) break;  // the counter only grows: every workgroup gets here
    while (j + 1 < m.njobs && t >= m.tile_base[j + 1]) ++j;
    const LdsArgs& a = m.jobs[j];
    const int32_t L = t - m.tile_base[j];
    const int32_t ttile = L / a.n_dtiles;
    dd_tile<D, M, WD, WT, CS, NLD, F, ES>(a, L - ttile * a.n_dtiles, ttile, lds);
  }
}

template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
hipError_t launch_multi(const MultiArgs& m, int32_t max_win, hipStream_t s) {
  constexpr int NT = 64 * WD * WT;
  if (!takes_rows<F, ES>()) return hipErrorInvalidValue;
  const size_t lds = tile_lds_bytes<CS, F>(max_win);
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
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(NT), lds, s, m);
  return hipGetLastError();
}

template <int D, int M, int WD, int WT, int CS, int NLD, int F, int ES>
hipError_t launch_one(const LdsArgs& a, hipStream_t s) {
  constexpr int NT = 64 * WD * WT;
  if (!takes_rows<F, ES>()) return hipErrorInvalidValue;
  const size_t lds = tile_lds_bytes<CS, F>(a.win);
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
  X(1, 4, 16, 1, 16, 3, 4)     \
  X(2, 2, 8, 1, 16, 4, 4)      \
  X(2, 2, 8, 1, 8, 2, 4)       \
  X(2, 2, 8, 1, 8, 2, 20)      \
  X(2, 2, 8, 1, 8, 2, 0)       \
  X(2, 2, 8, 1, 4, 1, 0)       \
  X(2, 2, 8, 1, 4, 1, 2)       \
  X(2, 2, 4, 1, 4, 2, 0)       \
  X(2, 2, 4, 1, 4, 2, 2)       \
  X(2, 1, 4, 1, 4, 1, 0)       \
  X(4, 1, 4, 1, 4, 2, 0)       \
  X(4, 1, 4, 1, 4, 2, 2)       \
  X(4, 1, 2, 2, 4, 2, 0)       \
  X(2, 2, 2, 1, 4, 3, 0)       \
  X(4, 1, 8, 1, 4, 1, 0)       \
  X(1, 4, 8, 1, 4, 2, 0)       \
  X(4, 1, 8, 2, 4, 1, 0)       \
  X(4, 1, 16, 1, 4, 1, 0)      \
  X(8, 1, 4, 1, 8, 4, 0)       \
  X(4, 2, 8, 1, 4, 1, 8)       \
  X(2, 2, 8, 1, 4, 1, 8)       \
  X(8, 1, 8, 1, 4, 1, 8)

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
