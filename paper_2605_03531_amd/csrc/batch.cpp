// Batched dedispersion + search of many chunks (beams) in one call: the
// chunks' corner turns and decimations, then one persistent dedispersion
// launch over the tiles of every (beam, DM range) job that shares an LDS tile
// shape and input element type, then each chunk's search. Optionally the whole sequence is captured
// once as a HIP graph and replayed while the batch's buffers stay the same.
#include <algorithm>
#include <cstring>
#include <list>
#include <mutex>

#include "k_dedisp_lds.h"
#include "sdd_internal.h"

namespace sdd {

namespace {
__global__ void k_zero_tickets(uint32_t* p, int32_t n) {
  if ((int32_t)threadIdx.x < n) p[threadIdx.x] = 0u;
}
}  // namespace

sdd_status launch_jobs_persistent(const std::vector<DedispArgs>& jobs, uint32_t* tickets,
                                  hipStream_t s) {
  // 8 tile counters per launch, zeroed by a kernel (no memset node in a
  // captured graph); one launch per group of jobs of one shape and element type
  hipLaunchKernelGGL(k_zero_tickets, dim3(1), dim3(kBatchTickets), 0, s, tickets,
                     (int32_t)kBatchTickets);
  SDD_HIP_TRY(hipGetLastError());
  int32_t launch = 0;
  std::vector<LdsArgs> la(jobs.size());
  std::vector<int> shape(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) shape[i] = lds_args_for(jobs[i], &la[i]);
  std::vector<char> done(jobs.size(), 0);
  for (size_t i = 0; i < jobs.size(); ++i) {
    if (done[i]) continue;
    if (shape[i] < 0) {
      done[i] = 1;
      SDD_HIP_TRY(launch_dedisperse(jobs[i], s));
      continue;
    }
    MultiArgs m{};
    int n = 0;
    int32_t tiles = 0, max_win = 0;
    for (size_t k = i; k < jobs.size() && n < kMaxJobs; ++k) {
      // one launch takes jobs of one shape and one element type (uint8 rows,
      // or the uint16 rows of decimated ranges)
      if (done[k] || shape[k] != shape[i] || la[k].es != la[i].es) continue;
      m.jobs[n] = la[k];
      m.tile_base[n] = tiles;
      tiles += la[k].n_dtiles * la[k].n_ttiles;
      max_win = std::max(max_win, la[k].win);
      done[k] = 1;
      ++n;
    }
    m.tile_base[n] = tiles;
    m.njobs = n;
    if (8 * (launch + 1) > kBatchTickets) {
      set_error("internal: more than %d persistent launches in one batch", kBatchTickets / 8);
      return SDD_EINVAL;
    }
    m.tickets = tickets + 8 * launch++;
    SDD_HIP_TRY(launch_dedisperse_lds_multi(m, max_win, shape[i], s));
  }
  return SDD_OK;
}

namespace {
int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }
}  // namespace

sdd_status batch_layout(const BatchJob* items, int32_t n, std::vector<ItemGeom>* out,
                        int64_t* total) {
  if (!items || n < 1) SDD_FAIL(SDD_EINVAL, "empty batch");
  out->assign(n, ItemGeom{});
  int64_t off = 0;
  for (int32_t k = 0; k < n; ++k) {
    const sdd_batch_item& it = items[k].it;
    if (!it.plan) SDD_FAIL(SDD_EINVAL, "item %d: null plan", k);
    if (it.plan->device != items[0].it.plan->device)
      SDD_FAIL(SDD_EINVAL, "item %d: all plans of a batch must use one device", k);
    ItemGeom& g = (*out)[k];
    sdd_status st = plan_geometry(it.plan, it.nsamp_in, &g.cg);
    if (st != SDD_OK) return st;
    g.ws_off = off;
    g.ws_bytes = it.d_planes ? g.cg.ws.total : g.cg.ws.total_planes;
    off = align256(off + g.ws_bytes);
  }
  // the persistent launch's tile counters after the items
  *total = off + align256(4 * kBatchTickets);
  return SDD_OK;
}

int64_t batch_tickets_off(const std::vector<ItemGeom>& geo) {
  const ItemGeom& g = geo.back();
  return align256(g.ws_off + g.ws_bytes);
}

namespace {

// ---- graph cache -----------------------------------------------------------

struct GraphEntry {
  std::vector<uint8_t> key;
  int device = 0;
  hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mu;
std::list<GraphEntry> g_graphs;  // most recently used first
constexpr size_t kMaxGraphs = 8;

void append(std::vector<uint8_t>& k, const void* p, size_t n) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  k.insert(k.end(), b, b + n);
}

std::vector<uint8_t> batch_key(const sdd_batch_item* items, int32_t n, int32_t flags,
                               const void* ws, hipStream_t s) {
  std::vector<uint8_t> k;
  append(k, &n, sizeof(n));
  append(k, &flags, sizeof(flags));
  append(k, &ws, sizeof(ws));
  append(k, &s, sizeof(s));
  for (int32_t i = 0; i < n; ++i) {
    const sdd_batch_item& it = items[i];
    append(k, &it.plan->id, sizeof(it.plan->id));
    append(k, &it.plan->version, sizeof(it.plan->version));
    sdd_batch_item c = it;
    c.plan = nullptr;
    c.d_planes = nullptr;
    c.plane_pitch = nullptr;
    append(k, &c, sizeof(c));
    const int32_t nr = (int32_t)it.plan->ranges.size();
    if (it.d_planes) {
      append(k, it.d_planes, sizeof(void*) * nr);
      append(k, it.plane_pitch, sizeof(int64_t) * nr);
    }
  }
  return k;
}

}  // namespace

sdd_status enqueue_batch(const BatchJob* items, int32_t n, int32_t flags,
                         std::vector<ItemGeom>& geo, uint8_t* ws, hipStream_t s) {
  std::vector<DedispArgs> jobs;
  for (int32_t k = 0; k < n; ++k) {
    const sdd_batch_item& it = items[k].it;
    ItemGeom& g = geo[k];
    uint8_t* iws = ws + g.ws_off;
    for (size_t r = 0; r < it.plan->ranges.size(); ++r) {
      if (it.d_planes) {
        g.planes[r] = it.d_planes[r];
        g.pitch[r] = it.plane_pitch[r];
      } else {
        g.planes[r] = reinterpret_cast<uint32_t*>(iws + g.cg.ws.plane_off[r]);
        g.pitch[r] = g.cg.ws.plane_pitch[r];
      }
    }
    std::vector<DedispArgs> own;
    sdd_status st = prep_item(it.plan, g.cg, it.d_in, it.nsamp_in, it.in_pitch, g.planes, g.pitch,
                              iws, s, (flags & SDD_BATCH_PER_ITEM) ? &own : &jobs,
                              items[k].ring_rows, items[k].ring_start);
    if (st != SDD_OK) return st;
    for (const auto& a : own) {
      StageTimer tm(SDD_STAGE_DEDISPERSE, s);
      SDD_HIP_TRY(launch_dedisperse(a, s));
    }
  }
  if (!(flags & SDD_BATCH_PER_ITEM)) {
    StageTimer tm(SDD_STAGE_DEDISPERSE, s);
    sdd_status st = launch_jobs_persistent(
        jobs, reinterpret_cast<uint32_t*>(ws + batch_tickets_off(geo)), s);
    if (st != SDD_OK) return st;
  }
  for (int32_t k = 0; k < n; ++k) {
    const sdd_batch_item& it = items[k].it;
    if (it.plan->widths.empty()) continue;
    ItemGeom& g = geo[k];
    sdd_status st = run_search(it.plan, g.cg, (const uint32_t* const*)g.planes, g.pitch,
                               it.d_best, it.d_stats, it.d_cands, it.cap, it.d_ncand,
                               ws + g.ws_off, s);
    if (st != SDD_OK) return st;
  }
  return SDD_OK;
}

}  // namespace sdd

using namespace sdd;

static std::vector<BatchJob> wrap(const sdd_batch_item* items, int32_t n) {
  std::vector<BatchJob> v;
  if (items)
    for (int32_t k = 0; k < n; ++k) v.push_back(BatchJob{items[k], 0, 0});
  return v;
}

extern "C" sdd_status sdd_batch_workspace_size(const sdd_batch_item* items, int32_t n,
                                               int64_t* bytes) {
  clear_error();
  if (!bytes) SDD_FAIL(SDD_EINVAL, "null output");
  std::vector<ItemGeom> geo;
  std::vector<BatchJob> jobs = wrap(items, n);
  return batch_layout(jobs.data(), n, &geo, bytes);
}

extern "C" sdd_status sdd_batch_dedisperse_search(const sdd_batch_item* items, int32_t n,
                                                  int32_t flags, void* d_ws, int64_t ws_bytes,
                                                  void* stream) {
  clear_error();
  std::vector<ItemGeom> geo;
  int64_t need = 0;
  std::vector<BatchJob> bj = wrap(items, n);
  sdd_status st = batch_layout(bj.data(), n, &geo, &need);
  if (st != SDD_OK) return st;
  if (!d_ws || ws_bytes < need)
    SDD_FAIL(SDD_ENOMEM, "batch workspace %lld bytes < %lld needed", (long long)ws_bytes,
             (long long)need);
  SDD_CHECK_WS_ALIGN(d_ws);
  for (int32_t k = 0; k < n; ++k) {
    const sdd_batch_item& it = items[k];
    if ((st = check_input(it.plan, it.d_in, it.nsamp_in, it.in_pitch)) != SDD_OK) return st;
    if (it.d_planes &&
        (st = check_planes(it.plan, geo[k].cg, (const void* const*)it.d_planes,
                           it.plane_pitch)) != SDD_OK)
      return st;
    if (!it.plan->widths.empty() &&
        (!it.d_best || !it.d_ncand || it.cap < 0 || (it.cap > 0 && !it.d_cands)))
      SDD_FAIL(SDD_EINVAL, "item %d: null best/ncand, or null candidates with cap > 0", k);
  }
  DeviceGuard dg(items[0].plan->device);
  if (!dg.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", items[0].plan->device);
  for (int32_t k = 0; k < n; ++k)
    if ((st = plan_upload(items[k].plan)) != SDD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)d_ws;
  if ((flags & SDD_BATCH_GRAPH) && s == nullptr)
    SDD_FAIL(SDD_EINVAL, "graph capture needs a created stream, not the null stream");
  if (!(flags & SDD_BATCH_GRAPH)) return enqueue_batch(bj.data(), n, flags, geo, ws, s);

  std::vector<uint8_t> key = batch_key(items, n, flags, d_ws, s);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it) {
    if (it->device == items[0].plan->device && it->key == key) {
      g_graphs.splice(g_graphs.begin(), g_graphs, it);
      SDD_HIP_TRY(hipGraphLaunch(g_graphs.front().exec, s));
      return SDD_OK;
    }
  }
  SDD_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  st = enqueue_batch(bj.data(), n, flags, geo, ws, s);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (st != SDD_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) SDD_FAIL(SDD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) SDD_FAIL(SDD_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  if (g_graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(g_graphs.back().exec);
    g_graphs.pop_back();
  }
  g_graphs.push_front(GraphEntry{std::move(key), items[0].plan->device, exec});
  SDD_HIP_TRY(hipGraphLaunch(exec, s));
  return SDD_OK;
}

extern "C" sdd_status sdd_batch_graph_clear(void) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto& g : g_graphs) (void)hipGraphExecDestroy(g.exec);
  g_graphs.clear();
  return SDD_OK;
}
