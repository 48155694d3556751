// Autotuner: for each DM range of a plan, times every tile shape of the built
// menu that fits the range on the device (synthetic input in the range's own
// element type: uint8 rows at decimation 1, uint16 sums of dec samples for a
// decimated range) and keeps the fastest. Results can be cached in a text file, one line per range shape:
//   <nchan> <ndm> <dec> <span32> <span64> <cols> <kind> <d> <wd> <wt> <ppl> <cs>
// where span32/span64 are the range's delay spans over DM tiles of 32 and 64
// trials and cols the plane width the tuning ran at.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sdd_internal.h"

namespace sdd {
namespace {

struct Key {
  int64_t v[6];
  bool operator==(const Key& o) const { return std::memcmp(v, o.v, sizeof(v)) == 0; }
};

Key range_key(const sdd_plan* p, int32_t r, int64_t cols) {
  return Key{{p->nchan, p->ranges[r].ndm(), p->ranges[r].dec, range_span(p, r, 32),
              range_span(p, r, 64), cols}};
}

struct Entry {
  Key k;
  sdd_tile t;
};

std::vector<Entry> read_cache(const char* path) {
  std::vector<Entry> out;
  if (!path) return out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  Entry e;
  long long v[12];
  while (std::fscanf(f, "%lld %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld %lld", &v[0],
                     &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &v[10],
                     &v[11]) == 12) {
    for (int i = 0; i < 6; ++i) e.k.v[i] = v[i];
    e.t = sdd_tile{(int32_t)v[6], (int32_t)v[7], (int32_t)v[8], (int32_t)v[9], (int32_t)v[10],
                   (int32_t)v[11]};
    out.push_back(e);
  }
  std::fclose(f);
  return out;
}

void append_cache(const char* path, const Entry& e) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%lld %lld %lld %lld %lld %lld %d %d %d %d %d %d\n", (long long)e.k.v[0],
               (long long)e.k.v[1], (long long)e.k.v[2], (long long)e.k.v[3], (long long)e.k.v[4],
               (long long)e.k.v[5], e.t.kind, e.t.dm_per_wave, e.t.waves_dm, e.t.waves_time,
               e.t.pairs_per_lane, e.t.chan_stage);
  std::fclose(f);
}

__device__ __forceinline__ uint32_t hash32(int64_t i, uint32_t seed) {
  uint32_t h = (uint32_t)i * 2654435761u ^ seed;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  return h;
}

// Synthetic rows: bytes, or uint16 values in [0, max_val] (a decimated
// range's sums), so the timed kernel sees inputs of the range's own type.
__global__ void k_fill_hash(uint8_t* p, int64_t n, uint32_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint8_t)hash32(i, seed);
}
__global__ void k_fill_hash16(uint16_t* p, int64_t n, uint32_t seed, uint32_t max_val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint16_t)(hash32(i, seed) % (max_val + 1u));
}

}  // namespace
}  // namespace sdd

using namespace sdd;

extern "C" sdd_status sdd_autotune(sdd_plan* p, int64_t nsamp_in, const char* cache_path,
                                   void* stream) {
  clear_error();
  if (!p) SDD_FAIL(SDD_EINVAL, "null plan");
  CallGeom cg;
  sdd_status st = plan_geometry(p, nsamp_in, &cg);
  if (st != SDD_OK) return st;
  std::vector<Entry> cache = read_cache(cache_path);
  DeviceGuard dg(p->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", p->device);
  if ((st = plan_upload(p)) != SDD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* x = nullptr;
  uint32_t* plane = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (x) (void)hipFree(x);
    if (plane) (void)hipFree(plane);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  for (size_t r = 0; r < p->ranges.size(); ++r) {
    Range& R = p->ranges[r];
    const int64_t cols = cg.g.plane_cols[r];
    const Key key = range_key(p, (int32_t)r, cols);
    bool hit = false;
    for (const auto& e : cache)
      if (e.k == key) {
        int32_t span = 0;
        if (check_tile_fits(p, (int32_t)r, e.t, &span) == SDD_OK) {
          R.tile = e.t;
          R.tile_span = span;
          p->version++;
          hit = true;
        }
        break;
      }
    clear_error();
    if (hit) continue;
    if (!x) {
      // room for the uint8 rows and for any range's uint16 rows (pitch
      // rounded to 128 samples as in the call workspace); the plane fits
      // every range
      int64_t row_bytes = nsamp_in;
      for (const auto& RR : p->ranges)
        if (RR.dec > 1)
          row_bytes = std::max<int64_t>(row_bytes, 2 * ((nsamp_in / RR.dec + 127) / 128 * 128));
      const int64_t nx = (int64_t)p->nchan * row_bytes;
      int64_t np = 0;
      for (size_t q = 0; q < p->ranges.size(); ++q)
        np = std::max<int64_t>(np, (int64_t)p->ranges[q].ndm() *
                                       ((cg.g.plane_cols[q] + 63) / 64 * 64));
      if (hipMalloc(&x, nx) != hipSuccess || hipMalloc(&plane, np * 4) != hipSuccess ||
          hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        SDD_FAIL(SDD_ENOMEM, "autotune buffers do not fit");
      }
    }
    // the range's input: uint8 rows, or uint16 rows of nsamp_in / dec samples
    const int es = R.dec == 1 ? 1 : 2;
    const int64_t xlen = nsamp_in / R.dec;
    const int64_t xpitch = es == 1 ? nsamp_in : (xlen + 127) / 128 * 128;
    if (cols + R.max_delay > xlen) continue;
    if (es == 1)
      hipLaunchKernelGGL(k_fill_hash, dim3(4096), dim3(256), 0, s, x,
                         (int64_t)p->nchan * xpitch, 12345u);
    else
      hipLaunchKernelGGL(k_fill_hash16, dim3(4096), dim3(256), 0, s,
                         reinterpret_cast<uint16_t*>(x), (int64_t)p->nchan * xpitch,
                         12345u + (uint32_t)r, (uint32_t)(255 * R.dec));
    float best_ms = 1e30f;
    sdd_tile best = R.tile;
    int32_t best_span = R.tile_span;
    for (const sdd_tile& t : tile_menu()) {
      int32_t span = 0;
      if (check_tile_fits(p, (int32_t)r, t, &span) != SDD_OK) continue;
      DedispArgs a{};
      a.x = x;
      a.elem_bytes = es;
      a.x_pitch = xpitch;
      a.x_len = xlen;
      a.nchan = p->nchan;
      a.delays = p->d_delays[r];
      a.ndm = R.ndm();
      a.plane = plane;
      a.plane_pitch = (cols + 63) / 64 * 64;
      a.cols = cols;
      a.max_val = 255 * R.dec;
      a.tile = t;
      a.span = span;
      a.max_delay = R.max_delay;
      if (launch_dedisperse(a, s) != hipSuccess) continue;  // warm-up
      (void)hipEventRecord(e0, s);
      const int reps = 2;
      for (int k = 0; k < reps; ++k) (void)launch_dedisperse(a, s);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) {
        cleanup();
        SDD_FAIL(SDD_EDEVICE, "autotune timing failed");
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
        best_span = span;
      }
    }
    clear_error();
    R.tile = best;
    R.tile_span = best_span;
    p->version++;
    append_cache(cache_path, Entry{key, best});
  }
  cleanup();
  return SDD_OK;
}
