// Candidate sifting after the single-pulse search (Section 2.1): square
// stencils in the DM-time plane remove redundant candidates of one event;
// density-based clustering (DBSCAN, Ester et al. 1996) of the survivors in
// the DM-time plane keeps each cluster's highest-S/N member.
//
// The candidate list stays on the device and its length is read there, so
// nothing returns to the host. One thread per candidate:
//   k_sift_load   coordinates: FP64 trial DM, window start in native samples
//   k_stencil     one stencil pass (alive_in -> alive_out)
//   k_core        neighbour counts -> core flags; union-find roots reset
//   k_union       core-core neighbours joined by lock-free union-find that
//                 always hangs the larger root under the smaller, so every
//                 component ends rooted at its smallest index
//   k_label       cluster of each point (core: its root; border: the root of
//                 its earliest core neighbour; noise: -1)
//   k_best        per cluster the best key (S/N order, then list order) and
//                 the member count, by integer atomics (order-free)
//   k_emit        one workgroup: kept flags -> exclusive scan -> output
// When the plan's DMs ascend with the candidate order, a candidate's
// neighbours lie in a contiguous run found by binary search (widened by a
// few ulps); every pair inside is then tested exactly as defined.
#include <cstring>

#include "sdd_internal.h"

namespace sdd {
namespace {

struct SiftArgs {
  const sdd_candidate* cands;
  const int32_t* ncand;
  int32_t cap;
  int32_t nranges;
  int32_t dm_offset[SDD_MAX_RANGES];
  int32_t ndm[SDD_MAX_RANGES];
  int32_t dec[SDD_MAX_RANGES];
  const double* dms;  // plan's trial DMs, global trial index
  int32_t dm_sorted;  // candidate order is DM order
  int32_t min_pts;
  double eps_dm;
  int64_t eps_t;
  // workspace arrays (cap entries each)
  double* dm;
  int64_t* t;
  float* snr;
  int32_t* alive[2];
  int32_t* core;
  int32_t* parent;
  int32_t* label;
  unsigned long long* best;
  int32_t* size;
  int32_t* n;  // min(*ncand, cap)
  sdd_candidate* out;
  int32_t* nout;
  int32_t* sizes;
};

__device__ inline int32_t count_of(const SiftArgs& a) { return *a.n; }

__device__ inline bool near_pair(const SiftArgs& a, int32_t p, int32_t q, double hd, int64_t ht) {
  const double dd = fabs(a.dm[q] - a.dm[p]);
  const int64_t dt = a.t[q] - a.t[p];
  return dd <= hd && (dt < 0 ? -dt : dt) <= ht;
}

// q better than p: higher S/N, or equal S/N and earlier in the list
__device__ inline bool better(const SiftArgs& a, int32_t q, int32_t p) {
  return a.snr[q] > a.snr[p] || (a.snr[q] == a.snr[p] && q < p);
}

// Candidates that may lie within hd of p in DM: [lo, hi).
__device__ inline void dm_window(const SiftArgs& a, int32_t n, int32_t p, double hd, int32_t* lo,
                                 int32_t* hi) {
  if (!a.dm_sorted) {
    *lo = 0;
    *hi = n;
    return;
  }
  const double c = a.dm[p];
  const double slack = 1e-12 * (fabs(c) + hd) + 1e-300;
  const double vlo = c - hd - slack, vhi = c + hd + slack;
  int32_t l = 0, h = p;  // first index with dm >= vlo
  while (l < h) {
    const int32_t m = (l + h) >> 1;
    if (a.dm[m] < vlo) l = m + 1; else h = m;
  }
  *lo = l;
  l = p + 1;
  h = n;  // first index with dm > vhi
  while (l < h) {
    const int32_t m = (l + h) >> 1;
    if (a.dm[m] <= vhi) l = m + 1; else h = m;
  }
  *hi = l;
}

__global__ __launch_bounds__(256) void k_sift_load(SiftArgs a) {
  const int32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p == 0) {
    const int32_t nc = *a.ncand;
    *a.n = nc < a.cap ? (nc < 0 ? 0 : nc) : a.cap;
  }
  const int32_t nc = *a.ncand;
  const int32_t n = nc < a.cap ? nc : a.cap;
  if (p >= n) return;
  const sdd_candidate c = a.cands[p];
  const int r = c.range;
  // an entry that names no trial of the plan takes no part (never kept)
  const bool ok = r >= 0 && r < a.nranges && c.dm_index >= 0 && c.dm_index < a.ndm[r];
  a.dm[p] = ok ? a.dms[a.dm_offset[r] + c.dm_index] : 0.0;
  a.t[p] = ok ? c.sample * (int64_t)a.dec[r] : 0;
  a.snr[p] = c.snr;
  a.alive[0][p] = ok ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_stencil(SiftArgs a, int src, double hd, int64_t ht) {
  const int32_t n = count_of(a);
  const int32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const int32_t* in = a.alive[src];
  int32_t keep = in[p];
  if (keep) {
    int32_t lo, hi;
    dm_window(a, n, p, hd, &lo, &hi);
    for (int32_t q = lo; q < hi; ++q)
      if (q != p && in[q] && near_pair(a, p, q, hd, ht) && better(a, q, p)) {
        keep = 0;
        break;
      }
  }
  a.alive[src ^ 1][p] = keep;
}

__global__ __launch_bounds__(256) void k_core(SiftArgs a, int src) {
  const int32_t n = count_of(a);
  const int32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const int32_t* in = a.alive[src];
  int32_t cnt = 0;
  if (in[p]) {
    int32_t lo, hi;
    dm_window(a, n, p, a.eps_dm, &lo, &hi);
    for (int32_t q = lo; q < hi; ++q)
      if (in[q] && near_pair(a, p, q, a.eps_dm, a.eps_t)) ++cnt;
  }
  a.core[p] = in[p] && cnt >= a.min_pts;
  a.parent[p] = p;
  a.best[p] = 0ull;
  a.size[p] = 0;
}

__device__ inline int32_t load_parent(const int32_t* par, int32_t x) {
  return __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t find_root(const int32_t* par, int32_t x) {
  // parents only ever decrease, so the walk ends at a root
  for (;;) {
    const int32_t y = load_parent(par, x);
    if (y == x) return x;
    x = y;
  }
}

__global__ __launch_bounds__(256) void k_union(SiftArgs a) {
  const int32_t n = count_of(a);
  const int32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n || !a.core[p]) return;
  int32_t lo, hi;
  dm_window(a, n, p, a.eps_dm, &lo, &hi);
  for (int32_t q = lo; q < p && q < hi; ++q) {
    if (!a.core[q] || !near_pair(a, p, q, a.eps_dm, a.eps_t)) continue;
    for (;;) {
      const int32_t rp = find_root(a.parent, p), rq = find_root(a.parent, q);
      if (rp == rq) break;
      const int32_t big = rp > rq ? rp : rq, small = rp > rq ? rq : rp;
      int32_t expect = big;
      // hang the larger root under the smaller one, unless it moved meanwhile
      if (__hip_atomic_compare_exchange_strong(a.parent + big, &expect, small, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        break;
    }
  }
}

__global__ __launch_bounds__(256) void k_label(SiftArgs a, int src) {
  const int32_t n = count_of(a);
  const int32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  int32_t lab = -1;
  if (a.alive[src][p]) {
    if (a.core[p]) {
      lab = find_root(a.parent, p);
    } else {
      int32_t lo, hi;
      dm_window(a, n, p, a.eps_dm, &lo, &hi);
      for (int32_t q = lo; q < hi; ++q)
        if (a.core[q] && near_pair(a, p, q, a.eps_dm, a.eps_t)) {
          lab = find_root(a.parent, q);
          break;
        }
    }
  }
  a.label[p] = lab;
}

__device__ inline unsigned long long sift_key(float snr, int32_t p) {
  uint32_t b;
  memcpy(&b, &snr, 4);
  if (b == 0x80000000u) b = 0u;  // -0 equals +0 as an S/N
  const uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // float order as uint
  return ((unsigned long long)ord << 32) | (uint32_t)(0xffffffffu - (uint32_t)p);
}

__global__ __launch_bounds__(256) void k_best(SiftArgs a) {
  const int32_t n = count_of(a);
  const int32_t p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const int32_t lab = a.label[p];
  if (lab < 0) return;
  atomicMax(a.best + lab, sift_key(a.snr[p], p));
  atomicAdd(a.size + lab, 1);
}

// One workgroup of 1024: kept flags in chunks, exclusive scan, output.
__global__ __launch_bounds__(1024) void k_emit(SiftArgs a, int src, int clustered) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry_s;
  const int32_t n = count_of(a);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (int32_t base = 0; base < n; base += 1024) {
    const int32_t p = base + tid;
    int32_t keep = 0, sz = 1;
    if (p < n) {
      if (clustered) {
        const int32_t lab = a.label[p];
        keep = lab >= 0 && a.best[lab] == sift_key(a.snr[p], p);
        if (keep) sz = a.size[lab];
      } else {
        keep = a.alive[src][p];
      }
    }
    const unsigned long long bal = __ballot(keep);
    const int32_t below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    int32_t off = carry_s, tot = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wid) off += wsum[w];
      tot += wsum[w];
    }
    if (keep) {
      const int32_t at = off + below;
      a.out[at] = a.cands[p];
      if (a.sizes) a.sizes[at] = sz;
    }
    __syncthreads();
    if (tid == 0) carry_s += tot;
    __syncthreads();
  }
  if (tid == 0) *a.nout = carry_s;
}

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

// Workspace: per entry dm f64, t i64, snr f32, two alive flags, core,
// parent, label, best u64, size (all cap long), then the count.
int64_t sift_ws_bytes(int32_t cap) {
  const int64_t c = cap;
  return align256(8 * c) * 3 + align256(4 * c) * 7 + 256;
}

}  // namespace

}  // namespace sdd

using namespace sdd;

extern "C" sdd_status sdd_sift_workspace_size(int32_t cap, int64_t* bytes) {
  clear_error();
  if (cap < 1 || !bytes) SDD_FAIL(SDD_EINVAL, "cap must be >= 1 and bytes non-null");
  *bytes = sift_ws_bytes(cap);
  return SDD_OK;
}

extern "C" sdd_status sdd_sift_candidates(const sdd_plan* plan, const sdd_candidate* d_cands,
                                          const int32_t* d_ncand, int32_t cap,
                                          const sdd_sift_desc* desc, sdd_candidate* d_out,
                                          int32_t* d_nout, int32_t* d_sizes, void* d_workspace,
                                          int64_t ws_bytes, void* stream) {
  clear_error();
  if (!plan || !d_cands || !d_ncand || !desc || !d_out || !d_nout || !d_workspace)
    SDD_FAIL(SDD_EINVAL, "null argument");
  if (cap < 1) SDD_FAIL(SDD_EINVAL, "cap must be >= 1");
  if (desc->nstencils < 0 || desc->nstencils > SDD_MAX_STENCILS)
    SDD_FAIL(SDD_EINVAL, "nstencils %d outside 0..%d", desc->nstencils, SDD_MAX_STENCILS);
  for (int k = 0; k < desc->nstencils; ++k)
    if (!(desc->stencil_dm[k] >= 0.0) || desc->stencil_t[k] < 0)
      SDD_FAIL(SDD_EINVAL, "stencil %d has a negative or NaN half-size", k);
  if (desc->min_pts < 0) SDD_FAIL(SDD_EINVAL, "min_pts must be >= 0");
  if (desc->min_pts > 0 && (!(desc->eps_dm >= 0.0) || desc->eps_t < 0))
    SDD_FAIL(SDD_EINVAL, "negative or NaN clustering neighbourhood");
  if (ws_bytes < sift_ws_bytes(cap))
    SDD_FAIL(SDD_ENOMEM, "sift workspace needs %lld bytes", (long long)sift_ws_bytes(cap));
  SDD_CHECK_WS_ALIGN(d_workspace);
  DeviceGuard dg(plan->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", plan->device);
  sdd_status st = plan_upload(plan);
  if (st != SDD_OK) return st;
  hipStream_t s = (hipStream_t)stream;

  SiftArgs a{};
  a.cands = d_cands;
  a.ncand = d_ncand;
  a.cap = cap;
  a.nranges = (int32_t)plan->ranges.size();
  bool sorted = true;
  double prev = -1.0;
  for (int r = 0; r < a.nranges; ++r) {
    const Range& R = plan->ranges[r];
    a.dm_offset[r] = R.dm_offset;
    a.ndm[r] = R.ndm();
    a.dec[r] = R.dec;
    for (double v : R.dms) {
      if (v < prev) sorted = false;
      prev = v;
    }
  }
  a.dms = plan->d_dms;
  a.dm_sorted = sorted ? 1 : 0;
  a.min_pts = desc->min_pts;
  a.eps_dm = desc->eps_dm;
  a.eps_t = desc->eps_t;
  uint8_t* w = (uint8_t*)d_workspace;
  const int64_t c = cap;
  a.dm = (double*)w;
  w += align256(8 * c);
  a.t = (int64_t*)w;
  w += align256(8 * c);
  a.best = (unsigned long long*)w;
  w += align256(8 * c);
  a.snr = (float*)w;
  w += align256(4 * c);
  a.alive[0] = (int32_t*)w;
  w += align256(4 * c);
  a.alive[1] = (int32_t*)w;
  w += align256(4 * c);
  a.core = (int32_t*)w;
  w += align256(4 * c);
  a.parent = (int32_t*)w;
  w += align256(4 * c);
  a.label = (int32_t*)w;
  w += align256(4 * c);
  a.size = (int32_t*)w;
  w += align256(4 * c);
  a.n = (int32_t*)w;
  a.out = d_out;
  a.nout = d_nout;
  a.sizes = d_sizes;

  StageTimer tm(SDD_STAGE_SIFT, s);
  const dim3 grid((unsigned)((cap + 255) / 256)), blk(256);
  hipLaunchKernelGGL(k_sift_load, grid, blk, 0, s, a);
  int src = 0;
  for (int k = 0; k < desc->nstencils; ++k) {
    hipLaunchKernelGGL(k_stencil, grid, blk, 0, s, a, src, desc->stencil_dm[k],
                       desc->stencil_t[k]);
    src ^= 1;
  }
  const int clustered = desc->min_pts > 0;
  if (clustered) {
    hipLaunchKernelGGL(k_core, grid, blk, 0, s, a, src);
    hipLaunchKernelGGL(k_union, grid, blk, 0, s, a);
    hipLaunchKernelGGL(k_label, grid, blk, 0, s, a, src);
    hipLaunchKernelGGL(k_best, grid, blk, 0, s, a);
  }
  hipLaunchKernelGGL(k_emit, dim3(1), dim3(1024), 0, s, a, src, clustered);
  SDD_HIP_TRY(hipGetLastError());
  return SDD_OK;
}
