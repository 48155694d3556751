// Input preparation kernels: corner turn of spectra-ordered input into
// channel rows, and exact time decimation (sums of consecutive samples,
// the downsampling of Section 3.2 applied before dedispersion).
#include "sdd_internal.h"

namespace sdd {
namespace {

constexpr int kCtChan = 64;    // channels per corner-turn tile
constexpr int kCtTime = 256;   // samples per corner-turn tile
constexpr int kCtPad = 4;

// in: byte (t, c) at in[t * in_pitch + c]; out: byte (c, t) at out[c * out_pitch + t].
// One workgroup turns a 256-sample x 64-channel tile through LDS: reads are
// rows of 64 channel bytes per spectrum, writes are rows of 256 sample bytes
// per channel (one full wavefront of dwords).
// With ring_rows > 0 the input is a ring of ring_rows spectra and sample t
// of the window is row (ring_start + t) mod ring_rows.
__global__ __launch_bounds__(256) void k_corner_turn(const uint8_t* __restrict__ in, int64_t nsamp,
                                                     int64_t in_pitch, int32_t nchan,
                                                     uint8_t* __restrict__ out, int64_t out_pitch,
                                                     int dword_in, int dword_out,
                                                     int64_t ring_rows, int64_t ring_start,
                                                     const uint8_t* __restrict__ lut,
                                                     const uint8_t* __restrict__ tmask) {
  __shared__ __attribute__((aligned(16))) uint8_t tile[kCtChan][kCtTime + kCtPad];
  const int tid = threadIdx.x;
  const int32_t c0 = blockIdx.y * kCtChan;
  const int64_t t0 = (int64_t)blockIdx.x * kCtTime;
  const int cc = (tid & 15) * 4;
#pragma unroll 4
  for (int k = 0; k < kCtTime / 16; ++k) {
    const int r = (tid >> 4) + 16 * k;
    const int64_t t = t0 + r;
    uint32_t v = 0;
    if (t < nsamp) {
      int64_t row = t;
      if (ring_rows > 0) {
        row = ring_start + t;
        row -= (row / ring_rows) * ring_rows;
      }
      const uint8_t* src = in + row * in_pitch + c0 + cc;
      if (dword_in && c0 + cc + 3 < nchan) {
        v = *reinterpret_cast<const uint32_t*>(src);
      } else {
        for (int b = 0; b < 4; ++b)
          if (c0 + cc + b < nchan) v |= (uint32_t)src[b] << (8 * b);
      }
    }
    tile[cc + 0][r] = (uint8_t)(v);
    tile[cc + 1][r] = (uint8_t)(v >> 8);
    tile[cc + 2][r] = (uint8_t)(v >> 16);
    tile[cc + 3][r] = (uint8_t)(v >> 24);
  }
  __syncthreads();
  const int tt = (tid & 63) * 4;
#pragma unroll 4
  for (int k = 0; k < kCtChan / 4; ++k) {
    const int cr = (tid >> 6) + 4 * k;
    const int32_t c = c0 + cr;
    const int64_t t = t0 + tt;
    if (c >= nchan || t >= nsamp) continue;
    uint8_t* dst = out + (int64_t)c * out_pitch + t;
    uint32_t v = *reinterpret_cast<const uint32_t*>(&tile[cr][tt]);
    if (lut || tmask) {
      // pre-conditioning: per-channel byte map, then the time mask
      uint32_t w = 0;
      for (int b = 0; b < 4; ++b) {
        uint32_t x = (v >> (8 * b)) & 255u;
        if (lut) x = lut[(int64_t)c * 256 + x];
        if (tmask && (t + b >= nsamp || !tmask[t + b])) x = 0;
        w |= x << (8 * b);
      }
      v = w;
    }
    if (dword_out && t + 3 < nsamp) {
      *reinterpret_cast<uint32_t*>(dst) = v;
    } else {
      for (int b = 0; b < 4 && t + b < nsamp; ++b) dst[b] = (uint8_t)(v >> (8 * b));
    }
  }
}

// Corner turn of 16-byte-aligned spectra (in_pitch and the base a multiple of
// 16, nchan a multiple of 128, no pre-conditioning maps): a workgroup turns
// 128 channels x 128 samples. Thread (g, q), g < 8, q < 32, loads 16
// channels (one 16-byte load) of each of the 4 spectra 4q..4q+3 (a wavefront
// reads 128 contiguous bytes of 8 spectra per load), turns each 4 x 4 byte
// block in registers (two rounds of v_perm) into words of 4 consecutive
// samples of one channel and stores them to LDS; then each thread writes 16
// samples of one channel (a wavefront writes 128 contiguous bytes of 8
// channel rows per store). LDS rows are 136 bytes, and the 16-byte blocks of
// row r are stored at block index b ^ (2 * ((r >> 5) & 3)): the word stores
// of a wavefront (8 groups 16 rows apart x 8 quads) then hit 64 different
// banks (rows alone would leave them on 16), and the row reads take whole
// rows, so they stay conflict-free. (The time did not change, 0.546 ms on
// the full-band chunk either way: HBM bounds the kernel.)
constexpr int kCtC = 128, kCtT = 128, kCtRow = kCtT + 8;
__global__ __launch_bounds__(256) void k_corner_turn128(const uint8_t* __restrict__ in,
                                                        int64_t nsamp, int64_t in_pitch,
                                                        uint8_t* __restrict__ out,
                                                        int64_t out_pitch, int64_t ring_rows,
                                                        int64_t ring_start) {
  __shared__ __attribute__((aligned(16))) uint8_t tile[kCtC * kCtRow];
  const int tid = threadIdx.x;
  const int g = tid & 7;          // 16-channel group
  const int q = tid >> 3;         // 4-sample quad, 0..31
  const int32_t c0 = blockIdx.y * kCtC;
  const int64_t t0 = (int64_t)blockIdx.x * kCtT;
  uint32_t w[4][4];               // [spectrum][word of 4 channels]
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t t = t0 + 4 * q + r;
    if (t < nsamp) {
      int64_t row = t;
      if (ring_rows > 0) {
        row = ring_start + t;
        row -= (row / ring_rows) * ring_rows;
      }
      const uint4 v = *reinterpret_cast<const uint4*>(in + row * in_pitch + c0 + 16 * g);
      w[r][0] = v.x; w[r][1] = v.y; w[r][2] = v.z; w[r][3] = v.w;
    } else {
      w[r][0] = w[r][1] = w[r][2] = w[r][3] = 0u;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // spectra 0..3 x channels 16g + 4k .. +3 -> one word of 4 samples per channel
    const uint32_t lo01 = __builtin_amdgcn_perm(w[1][k], w[0][k], 0x05010400u);
    const uint32_t hi01 = __builtin_amdgcn_perm(w[1][k], w[0][k], 0x07030602u);
    const uint32_t lo23 = __builtin_amdgcn_perm(w[3][k], w[2][k], 0x05010400u);
    const uint32_t hi23 = __builtin_amdgcn_perm(w[3][k], w[2][k], 0x07030602u);
    const uint32_t ch[4] = {__builtin_amdgcn_perm(lo23, lo01, 0x05040100u),
                            __builtin_amdgcn_perm(lo23, lo01, 0x07060302u),
                            __builtin_amdgcn_perm(hi23, hi01, 0x05040100u),
                            __builtin_amdgcn_perm(hi23, hi01, 0x07060302u)};
#pragma unroll
    for (int b = 0; b < 4; ++b)
    {
      const int r = 16 * g + 4 * k + b;
      *reinterpret_cast<uint32_t*>(tile + r * kCtRow + 16 * ((q >> 2) ^ (((r >> 5) & 3) << 1)) +
                                   4 * (q & 3)) = ch[b];
    }
  }
  __syncthreads();
  // 128 channels x 8 pieces of 16 samples: thread takes pieces tid + 256 p
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int e = tid + 256 * p;
    const int c = e >> 3, sp = e & 7;
    const int64_t t = t0 + 16 * sp;
    const uint2* src =
        reinterpret_cast<const uint2*>(tile + c * kCtRow + 16 * (sp ^ (((c >> 5) & 3) << 1)));
    const uint2 a = src[0], b = src[1];
    uint8_t* dst = out + (int64_t)(c0 + c) * out_pitch + t;
    if (t + 16 <= nsamp) {
      *reinterpret_cast<uint4*>(dst) = make_uint4(a.x, a.y, b.x, b.y);
    } else {
      const uint32_t v[4] = {a.x, a.y, b.x, b.y};
      for (int k2 = 0; k2 < 16 && t + k2 < nsamp; ++k2) dst[k2] = (uint8_t)(v[k2 >> 2] >> (8 * (k2 & 3)));
    }
  }
}

// Channel rows through the pre-conditioning maps: 4 samples per thread.
__global__ __launch_bounds__(256) void k_precond_rows(const uint8_t* __restrict__ in,
                                                      int64_t in_pitch, int64_t nsamp,
                                                      int32_t nchan,
                                                      const uint8_t* __restrict__ lut,
                                                      const uint8_t* __restrict__ tmask,
                                                      uint8_t* __restrict__ out,
                                                      int64_t out_pitch) {
  const int64_t t = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (t >= nsamp) return;
  for (int32_t c = blockIdx.y; c < nchan; c += gridDim.y) {
    const uint8_t* src = in + (int64_t)c * in_pitch;
    uint8_t* dst = out + (int64_t)c * out_pitch;
    for (int b = 0; b < 4 && t + b < nsamp; ++b) {
      uint32_t x = src[t + b];
      if (lut) x = lut[(int64_t)c * 256 + x];
      if (tmask && !tmask[t + b]) x = 0;
      dst[t + b] = (uint8_t)x;
    }
  }
}

template <typename Tin>
__global__ __launch_bounds__(256) void k_decimate(const Tin* __restrict__ in, int64_t in_pitch,
                                                  int32_t nchan, int32_t factor,
                                                  uint16_t* __restrict__ out, int64_t out_pitch,
                                                  int64_t out_len) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= out_len) return;
  for (int32_t c = blockIdx.y; c < nchan; c += gridDim.y) {
    const Tin* src = in + (int64_t)c * in_pitch + j * factor;
    uint32_t s = 0;
    for (int k = 0; k < factor; ++k) s += src[k];
    out[(int64_t)c * out_pitch + j] = (uint16_t)s;
  }
}

// Every power-of-two decimation up to 16 of uint8 rows in one pass. A thread
// owns 16 consecutive samples (one 16-byte load), forms the exact pairwise
// sums level by level (2, 4, 8, 16 samples) and writes the levels the plan
// uses; a wavefront's writes of one level are contiguous. Each input byte is
// read once; each level's rows are written once (1 + 2 * sum 1/dec bytes of
// traffic per input byte, against the pass-per-level form that re-reads every
// level it builds from).
__global__ __launch_bounds__(256) void k_decimate_pow2(const uint8_t* __restrict__ in,
                                                       int64_t in_pitch, int64_t nsamp,
                                                       int32_t nchan, int vec, DecLevels lv) {
  const int64_t t = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
  if (t >= nsamp) return;
  for (int32_t c = blockIdx.y; c < nchan; c += gridDim.y) {
    const uint8_t* src = in + (int64_t)c * in_pitch + t;
    uint32_t w[4];
    if (vec && t + 16 <= nsamp) {
      const uint4 v = *reinterpret_cast<const uint4*>(src);
      w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else {
      // samples past the row end read as 0; no output that uses them is written
      for (int q = 0; q < 4; ++q) w[q] = 0u;
      for (int b = 0; b < 16 && t + b < nsamp; ++b) w[b >> 2] |= (uint32_t)src[b] << (8 * (b & 3));
    }
    // level 1: sums of 2 samples, as packed 16-bit pairs (s1[q] = outputs 2q, 2q+1)
    uint32_t s1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      s1[q] = ((w[q] & 0xffu) + ((w[q] >> 8) & 0xffu)) |
              ((((w[q] >> 16) & 0xffu) + (w[q] >> 24)) << 16);
    uint32_t s2[2], s3, s4;
#pragma unroll
    for (int q = 0; q < 2; ++q)
      s2[q] = ((s1[2 * q] & 0xffffu) + (s1[2 * q] >> 16)) |
              (((s1[2 * q + 1] & 0xffffu) + (s1[2 * q + 1] >> 16)) << 16);
    s3 = ((s2[0] & 0xffffu) + (s2[0] >> 16)) | (((s2[1] & 0xffffu) + (s2[1] >> 16)) << 16);
    s4 = (s3 & 0xffffu) + (s3 >> 16);
    // level l holds 16 >> l outputs starting at output t >> l
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      uint16_t* o = lv.out[l];
      if (!o) continue;
      const int n = 8 >> l;                   // outputs of this thread at level l
      const int64_t j0 = t >> (l + 1);
      uint16_t* dst = o + (int64_t)c * lv.pitch[l] + j0;
      const uint32_t* vals = l == 0 ? s1 : l == 1 ? s2 : l == 2 ? &s3 : &s4;
      if (lv.vec[l] && j0 + n <= lv.len[l]) {
        if (l == 0)
          *reinterpret_cast<uint4*>(dst) = make_uint4(s1[0], s1[1], s1[2], s1[3]);
        else if (l == 1)
          *reinterpret_cast<uint2*>(dst) = make_uint2(s2[0], s2[1]);
        else if (l == 2)
          *reinterpret_cast<uint32_t*>(dst) = s3;
        else
          *dst = (uint16_t)s4;
      } else {
        for (int k = 0; k < n && j0 + k < lv.len[l]; ++k)
          dst[k] = (uint16_t)(vals[k >> 1] >> (16 * (k & 1)));
      }
    }
  }
}

}  // namespace

hipError_t launch_decimate_pow2(const uint8_t* in, int64_t in_pitch, int64_t nsamp, int32_t nchan,
                                const DecLevels& lv, hipStream_t s) {
  DecLevels l = lv;
  for (int k = 0; k < 4; ++k) {
    const int bytes = 16 >> k;  // bytes of one thread's outputs at level k
    l.vec[k] = l.out[k] && ((uintptr_t)l.out[k] % bytes == 0) && ((l.pitch[k] * 2) % bytes == 0);
  }
  const int vec = ((uintptr_t)in % 16 == 0) && (in_pitch % 16 == 0);
  dim3 grid((unsigned)((nsamp + 4095) / 4096), (unsigned)(nchan < 1024 ? nchan : 1024));
  hipLaunchKernelGGL(k_decimate_pow2, grid, dim3(256), 0, s, in, in_pitch, nsamp, nchan, vec, l);
  return hipGetLastError();
}

hipError_t launch_corner_turn(const uint8_t* in, int64_t nsamp, int64_t in_pitch, int32_t nchan,
                              uint8_t* out, int64_t out_pitch, hipStream_t s, int64_t ring_rows,
                              int64_t ring_start, const uint8_t* lut, const uint8_t* tmask) {
  if (!lut && !tmask && nchan % kCtC == 0 && (uintptr_t)in % 16 == 0 && in_pitch % 16 == 0 &&
      (uintptr_t)out % 16 == 0 && out_pitch % 16 == 0) {
    dim3 grid((unsigned)((nsamp + kCtT - 1) / kCtT), (unsigned)(nchan / kCtC));
    hipLaunchKernelGGL(k_corner_turn128, grid, dim3(256), 0, s, in, nsamp, in_pitch, out,
                       out_pitch, ring_rows, ring_start);
    return hipGetLastError();
  }
  const int dword_in = ((uintptr_t)in % 4 == 0) && (in_pitch % 4 == 0);
  const int dword_out = ((uintptr_t)out % 4 == 0) && (out_pitch % 4 == 0);
  dim3 grid((unsigned)((nsamp + kCtTime - 1) / kCtTime), (unsigned)((nchan + kCtChan - 1) / kCtChan));
  hipLaunchKernelGGL(k_corner_turn, grid, dim3(256), 0, s, in, nsamp, in_pitch, nchan, out,
                     out_pitch, dword_in, dword_out, ring_rows, ring_start, lut, tmask);
  return hipGetLastError();
}

hipError_t launch_precond_rows(const uint8_t* in, int64_t in_pitch, int64_t nsamp, int32_t nchan,
                               const uint8_t* lut, const uint8_t* tmask, uint8_t* out,
                               int64_t out_pitch, hipStream_t s) {
  dim3 grid((unsigned)((nsamp + 1023) / 1024), (unsigned)(nchan < 65535 ? nchan : 65535));
  hipLaunchKernelGGL(k_precond_rows, grid, dim3(256), 0, s, in, in_pitch, nsamp, nchan, lut, tmask,
                     out, out_pitch);
  return hipGetLastError();
}

hipError_t launch_decimate(const void* in, int in_bytes, int64_t in_pitch, int32_t nchan,
                           int32_t factor, uint16_t* out, int64_t out_pitch, int64_t out_len,
                           hipStream_t s) {
  dim3 grid((unsigned)((out_len + 255) / 256), (unsigned)(nchan < 1024 ? nchan : 1024));
  if (in_bytes == 1)
    hipLaunchKernelGGL(k_decimate<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)in, in_pitch,
                       nchan, factor, out, out_pitch, out_len);
  else
    hipLaunchKernelGGL(k_decimate<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)in,
                       in_pitch, nchan, factor, out, out_pitch, out_len);
  return hipGetLastError();
}

}  // namespace sdd
