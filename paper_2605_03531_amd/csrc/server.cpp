// Streaming server: many beams arriving as chunks of spectra, dedispersed and
// searched with continuous batching on one GPU.
//
// Each open stream (beam) owns a device ring of time-major spectra, R rows of
// nchan bytes, R a multiple of the chunk length N and at least overlap + 2N.
// Submitting chunk s copies it to rows [sN, (s+1)N) mod R; output chunk k
// (owned native samples [kN, (k+1)N)) becomes ready once samples below
// (k+1)N + O are present, O the plan's overlap. This is the device-side
// counterpart of the paper's host ring buffer of recent spectra (Section 2.2):
// its depth absorbs the pipeline delay.
//
// A scheduler thread packs ready chunks from any streams (oldest first, at
// most max_batch) into one batch and runs it on a free slot: a HIP stream with
// its own workspace and result buffers. Chunks that become ready while other
// batches run join the next batch. A completer thread waits for each batch,
// copies its per-DM best values and candidates into host memory and queues
// the results for sdd_stream_poll.
//
// Admission: sdd_stream_open refuses (SDD_EAGAIN) a beam whose ring, plus the
// slot workspaces grown for it, would exceed the HBM budget. Backpressure:
// sdd_stream_submit refuses (SDD_EAGAIN) a chunk that would overwrite ring
// rows an unfinished output chunk still needs.
//
// With SDD_SERVER_FAKE the server allocates no device memory and runs no
// kernel: a batch just sleeps fake_exec_us and yields empty results. The
// scheduling, admission and backpressure logic is the same, so it can be
// tested without a GPU.
#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "sdd_internal.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

struct WorkItem {
  sdd_stream* st;
  int64_t k;          // output chunk
  int64_t t_ready;
  bool keep = false;  // write the planes into `planes` (a kept-planes stream)
  uint8_t* planes = nullptr;  // device buffer of the chunk's planes, all ranges
};

struct ResultBox {
  sdd_result r{};
  std::vector<sdd_dm_best> best;
  std::vector<sdd_candidate> cands;
  uint8_t* planes = nullptr;  // device memory behind r.d_planes (freed on release)
};

}  // namespace

struct sdd_stream {
  sdd_server* srv = nullptr;
  const sdd_plan* plan = nullptr;
  uint64_t tag = 0;
  int64_t N = 0, O = 0, R = 0;
  uint8_t* ring = nullptr;
  hipStream_t copy_stream = nullptr;
  int64_t submitted = 0;      // chunks written
  int64_t next_out = 0;       // next output chunk to schedule
  int64_t inflight = 0;       // scheduled, not completed
  int64_t oldest_pending = 0; // lowest output chunk not yet completed
  std::map<int64_t, int64_t> done_flags;  // completed chunks above oldest_pending
  std::deque<std::pair<int64_t, int64_t>> submit_times;  // (seq, ns)
  bool closing = false;
  bool frozen = false;        // a snapshot is reading the ring: schedule nothing
  bool keep_planes = false;   // output chunks also return their planes
  int64_t ring_bytes = 0;
  int64_t item_ws = 0;        // workspace bytes of one of its chunks
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t* ws = nullptr;
  int64_t ws_cap = 0;
  uint8_t* dout = nullptr;    // device results of the batch
  uint8_t* hout = nullptr;    // pinned host copy
  int64_t out_cap = 0;
  bool busy = false;
  bool launched = false;      // the batch's work and event are enqueued
  int64_t t_start = 0;
  std::vector<WorkItem> items;
  std::vector<int64_t> out_off;  // per item: offset of best, cands, ncand blocks
  int32_t status = SDD_OK;       // enqueue status of the batch
};

struct sdd_server {
  sdd_server_desc d{};
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_poll;
  bool stop = false;
  std::vector<sdd_stream*> streams;
  std::vector<Slot> slots;
  std::deque<ResultBox*> results;
  std::map<void*, ResultBox*> out_results;  // handed to the caller, not released
  int64_t hbm_used = 0;
  int64_t slot_item_ws = 0;   // per-item workspace the slots are sized for
  int64_t batches = 0, chunks = 0;
  double busy_ms = 0.0;
  std::thread th_sched, th_done;
  size_t rr = 0;              // round-robin start among streams
};

using namespace sdd;

namespace {

bool fake(const sdd_server* s) { return (s->d.flags & SDD_SERVER_FAKE) != 0; }

int64_t result_bytes(const sdd_plan* p, int32_t cap) {
  return align256((int64_t)p->ndm_total * sizeof(sdd_dm_best)) +
         align256((int64_t)cap * sizeof(sdd_candidate)) + 256;
}

// Plane layout of one output chunk (the workspace's plane pitches, ranges back
// to back at 256-byte offsets); returns the bytes, or -1.
int64_t chunk_planes(const sdd_plan* p, int64_t N, int64_t off[SDD_MAX_RANGES],
                     int64_t pitch[SDD_MAX_RANGES], int64_t cols[SDD_MAX_RANGES]) {
  CallGeom cg;
  if (plan_geometry(p, N + p->overlap, &cg) != SDD_OK) return -1;
  int64_t b = 0;
  for (int r = 0; r < (int)p->ranges.size(); ++r) {
    off[r] = b;
    pitch[r] = cg.ws.plane_pitch[r];
    cols[r] = cg.g.plane_cols[r];
    b = align256(b + (int64_t)p->ranges[r].ndm() * pitch[r] * 4);
  }
  return b;
}

void free_box(sdd_server* s, ResultBox* b) {
  if (b->planes && !fake(s)) {
    DeviceGuard g(s->d.device);
    (void)hipFree(b->planes);
  }
  delete b;
}

int64_t item_workspace(const sdd_plan* p, int64_t N) {
  CallGeom cg;
  if (plan_geometry(p, N + p->overlap, &cg) != SDD_OK) return -1;
  return align256(cg.ws.total_planes);
}

// Bytes a slot needs for max_batch chunks of item_ws each.
int64_t slot_ws_bytes(const sdd_server* s, int64_t item_ws) {
  // items, then the persistent launch's tile counters
  return (int64_t)s->d.max_batch * align256(item_ws) + align256(4 * kBatchTickets);
}

bool chunk_ready(const sdd_stream* st, int64_t k) {
  return st->submitted * st->N >= (k + 1) * st->N + st->O;
}

int64_t ready_time(const sdd_stream* st, int64_t k) {
  // the submit that made output chunk k complete
  const int64_t need = ((k + 1) * st->N + st->O + st->N - 1) / st->N - 1;
  for (const auto& p : st->submit_times)
    if (p.first == need) return p.second;
  return now_ns();
}

// Grows every slot to hold chunks of item_ws bytes. Caller holds s->mu and
// no slot is busy or the slots are only grown while idle.
sdd_status grow_slots_locked(sdd_server* s, int64_t item_ws, int64_t out_bytes) {
  for (auto& sl : s->slots) {
    const int64_t need = slot_ws_bytes(s, item_ws);
    const int64_t need_out = (int64_t)s->d.max_batch * out_bytes;
    if (sl.ws_cap < need) {
      if (!fake(s)) {
        if (sl.ws) SDD_HIP_TRY(hipFree(sl.ws));
        sl.ws = nullptr;
        SDD_HIP_TRY(hipMalloc(&sl.ws, need));
      }
      s->hbm_used += need - sl.ws_cap;
      sl.ws_cap = need;
    }
    if (sl.out_cap < need_out) {
      if (!fake(s)) {
        if (sl.dout) SDD_HIP_TRY(hipFree(sl.dout));
        if (sl.hout) SDD_HIP_TRY(hipHostFree(sl.hout));
        sl.dout = nullptr;
        sl.hout = nullptr;
        SDD_HIP_TRY(hipMalloc(&sl.dout, need_out));
        SDD_HIP_TRY(hipHostMalloc(&sl.hout, need_out, hipHostMallocDefault));
      }
      s->hbm_used += need_out - sl.out_cap;
      sl.out_cap = need_out;
    }
  }
  return SDD_OK;
}

void scheduler(sdd_server* s) {
  if (!fake(s)) (void)hipSetDevice(s->d.device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    // a free slot and ready work?
    Slot* slot = nullptr;
    for (auto& sl : s->slots)
      if (!sl.busy) {
        slot = &sl;
        break;
      }
    std::vector<WorkItem> batch;
    if (slot) {
      // oldest ready chunks first, round-robin among streams for ties
      const size_t ns = s->streams.size();
      for (int round = 0; (int)batch.size() < s->d.max_batch; ++round) {
        bool any = false;
        for (size_t q = 0; q < ns && (int)batch.size() < s->d.max_batch; ++q) {
          sdd_stream* st = s->streams[(s->rr + q) % ns];
          if (st->closing || st->frozen || !chunk_ready(st, st->next_out)) continue;
          batch.push_back(WorkItem{st, st->next_out, ready_time(st, st->next_out),
                                   st->keep_planes && !fake(s), nullptr});
          st->next_out++;
          st->inflight++;
          any = true;
        }
        if (!any) break;
      }
      if (ns) s->rr = (s->rr + 1) % ns;
    }
    if (batch.empty()) {
      s->cv_sched.wait(lk);
      continue;
    }
    slot->busy = true;
    slot->launched = false;
    slot->items = batch;
    slot->t_start = now_ns();
    s->batches++;
    s->chunks += (int64_t)batch.size();
    const int64_t batch_no = s->batches;
    lk.unlock();

    sdd_status st = SDD_OK;
    // fake mode: every fake_fail_every-th batch fails as a device error would
    if (fake(s) && s->d.fake_fail_every > 0 && batch_no % s->d.fake_fail_every == 0) {
      set_error("injected batch failure (batch %lld)", (long long)batch_no);
      st = SDD_EDEVICE;
    }
    if (!fake(s)) {
      std::vector<BatchJob> jobs(batch.size());
      // kept planes: one device buffer per chunk, handed to its result
      std::vector<std::array<uint32_t*, SDD_MAX_RANGES>> pptr(batch.size());
      std::vector<std::array<int64_t, SDD_MAX_RANGES>> ppitch(batch.size());
      slot->out_off.assign(batch.size(), 0);
      int64_t oo = 0;
      for (size_t q = 0; q < batch.size() && st == SDD_OK; ++q) {
        if (!slot->items[q].keep) continue;
        const sdd_stream* bs = batch[q].st;
        int64_t off[SDD_MAX_RANGES], cols[SDD_MAX_RANGES];
        const int64_t bytes = chunk_planes(bs->plan, bs->N, off, ppitch[q].data(), cols);
        void* buf = nullptr;
        if (bytes <= 0 || hipMalloc(&buf, bytes) != hipSuccess) {
          set_error("plane buffer of %lld bytes could not be allocated", (long long)bytes);
          st = SDD_ENOMEM;
          break;
        }
        slot->items[q].planes = static_cast<uint8_t*>(buf);
        for (int r = 0; r < (int)bs->plan->ranges.size(); ++r)
          pptr[q][r] = reinterpret_cast<uint32_t*>(slot->items[q].planes + off[r]);
      }
      for (size_t q = 0; q < batch.size(); ++q) {
        const sdd_stream* bs = batch[q].st;
        const sdd_plan* p = bs->plan;
        BatchJob& j = jobs[q];
        std::memset(&j.it, 0, sizeof(j.it));
        j.it.plan = p;
        if (slot->items[q].planes) {
          j.it.d_planes = pptr[q].data();
          j.it.plane_pitch = ppitch[q].data();
        }
        j.it.d_in = bs->ring;
        j.it.nsamp_in = bs->N + bs->O;
        j.it.in_pitch = p->nchan;
        j.ring_rows = bs->R;
        j.ring_start = (batch[q].k * bs->N) % bs->R;
        slot->out_off[q] = oo;
        uint8_t* o = slot->dout + oo;
        j.it.d_best = reinterpret_cast<sdd_dm_best*>(o);
        j.it.d_cands = reinterpret_cast<sdd_candidate*>(
            o + align256((int64_t)p->ndm_total * sizeof(sdd_dm_best)));
        j.it.cap = s->d.cap;
        j.it.d_ncand = reinterpret_cast<int32_t*>(
            o + align256((int64_t)p->ndm_total * sizeof(sdd_dm_best)) +
            align256((int64_t)s->d.cap * sizeof(sdd_candidate)));
        oo += result_bytes(p, s->d.cap);
      }
      std::vector<ItemGeom> geo;
      int64_t need = 0;
      if (st == SDD_OK) st = batch_layout(jobs.data(), (int32_t)jobs.size(), &geo, &need);
      if (st == SDD_OK && need > slot->ws_cap) {
        set_error("internal: slot workspace %lld < %lld", (long long)slot->ws_cap,
                  (long long)need);
        st = SDD_ENOMEM;
      }
      if (st == SDD_OK)
        st = enqueue_batch(jobs.data(), (int32_t)jobs.size(), s->d.batch_flags & SDD_BATCH_PER_ITEM,
                           geo, slot->ws, slot->stream);
      if (st == SDD_OK && hipMemcpyAsync(slot->hout, slot->dout, oo, hipMemcpyDeviceToHost,
                                         slot->stream) != hipSuccess)
        st = SDD_EDEVICE;
      if (hipEventRecord(slot->done, slot->stream) != hipSuccess && st == SDD_OK) st = SDD_EDEVICE;
    }
    lk.lock();
    slot->status = st;
    slot->launched = true;
    s->cv_done.notify_all();
  }
}

void completer(sdd_server* s) {
  if (!fake(s)) (void)hipSetDevice(s->d.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    Slot* slot = nullptr;
    for (auto& sl : s->slots)
      if (sl.busy && sl.launched && (!slot || sl.t_start < slot->t_start)) slot = &sl;
    if (!slot) {
      if (s->stop) break;
      s->cv_done.wait(lk);
      continue;
    }
    int32_t status = slot->status;
    lk.unlock();
    if (fake(s)) {
      std::this_thread::sleep_for(std::chrono::microseconds(s->d.fake_exec_us));
    } else if (status == SDD_OK && hipEventSynchronize(slot->done) != hipSuccess) {
      status = SDD_EDEVICE;
    } else if (status != SDD_OK) {
      (void)hipStreamSynchronize(slot->stream);
    }
    const int64_t t_done = now_ns();
    std::vector<ResultBox*> boxes;
    for (size_t q = 0; q < slot->items.size(); ++q) {
      const WorkItem& w = slot->items[q];
      const sdd_plan* p = w.st->plan;
      ResultBox* b = new ResultBox();
      b->best.assign(p->ndm_total, sdd_dm_best{});
      int32_t n = 0;
      if (!fake(s) && status == SDD_OK) {
        const uint8_t* h = slot->hout + slot->out_off[q];
        std::memcpy(b->best.data(), h, sizeof(sdd_dm_best) * p->ndm_total);
        const uint8_t* hc = h + align256((int64_t)p->ndm_total * sizeof(sdd_dm_best));
        std::memcpy(&n, hc + align256((int64_t)s->d.cap * sizeof(sdd_candidate)), sizeof(n));
        b->cands.resize(std::min(n, s->d.cap));
        std::memcpy(b->cands.data(), hc, sizeof(sdd_candidate) * b->cands.size());
      }
      sdd_result& r = b->r;
      b->planes = w.planes;
      if (w.planes && status == SDD_OK) {
        int64_t off[SDD_MAX_RANGES];
        chunk_planes(p, w.st->N, off, r.plane_pitch, r.plane_cols);
        r.nplanes = (int32_t)p->ranges.size();
        for (int q2 = 0; q2 < r.nplanes; ++q2) {
          r.d_planes[q2] = reinterpret_cast<const uint32_t*>(w.planes + off[q2]);
          r.plane_rows[q2] = p->ranges[q2].ndm();
        }
      }
      r.tag = w.st->tag;
      r.chunk = w.k;
      r.status = status;
      r.ncand = n;
      r.ndm = p->ndm_total;
      r.best = b->best.data();
      r.cands = b->cands.data();
      r.t_ready_ns = w.t_ready;
      r.t_start_ns = slot->t_start;
      r.t_done_ns = t_done;
      r.handle = b;
      boxes.push_back(b);
    }
    lk.lock();
    s->busy_ms += (t_done - slot->t_start) * 1e-6;
    for (size_t q = 0; q < slot->items.size(); ++q) {
      sdd_stream* st = slot->items[q].st;
      st->inflight--;
      st->done_flags[slot->items[q].k] = 1;
      while (st->done_flags.count(st->oldest_pending)) {
        st->done_flags.erase(st->oldest_pending);
        st->oldest_pending++;
      }
      s->results.push_back(boxes[q]);
    }
    slot->busy = false;
    slot->launched = false;
    slot->items.clear();
    s->cv_poll.notify_all();
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" sdd_status sdd_server_create(const sdd_server_desc* desc, sdd_server** out) {
  clear_error();
  if (!desc || !out) SDD_FAIL(SDD_EINVAL, "null argument");
  *out = nullptr;
  sdd_server_desc d = *desc;
  if (d.nstreams < 1 || d.nstreams > 16) SDD_FAIL(SDD_EINVAL, "nstreams must be in [1, 16]");
  if (d.max_batch < 1 || d.max_batch > 256) SDD_FAIL(SDD_EINVAL, "max_batch must be in [1, 256]");
  if (d.max_beams < 1) SDD_FAIL(SDD_EINVAL, "max_beams must be >= 1");
  if (d.hbm_budget <= 0) SDD_FAIL(SDD_EINVAL, "hbm_budget must be > 0");
  if (d.ring_chunks < 2) d.ring_chunks = 2;
  if (d.cap < 0) SDD_FAIL(SDD_EINVAL, "cap must be >= 0");
  if (d.device < 0) SDD_FAIL(SDD_EINVAL, "bad device");
  auto s = std::make_unique<sdd_server>();
  s->d = d;
  s->slots.resize(d.nstreams);
  if (!fake(s.get())) {
    DeviceGuard g(d.device);
    if (!g.ok) SDD_FAIL(SDD_EDEVICE, "cannot select device %d", d.device);
    for (auto& sl : s->slots) {
      SDD_HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
      SDD_HIP_TRY(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    }
  }
  sdd_server* raw = s.release();
  raw->th_sched = std::thread(scheduler, raw);
  raw->th_done = std::thread(completer, raw);
  *out = raw;
  return SDD_OK;
}

extern "C" sdd_status sdd_stream_footprint(const sdd_server* s, const sdd_plan* p,
                                           int64_t chunk_nsamp, int64_t* bytes) {
  clear_error();
  if (!s || !p || !bytes) SDD_FAIL(SDD_EINVAL, "null argument");
  if (chunk_nsamp < 1 || chunk_nsamp % p->dec_max != 0)
    SDD_FAIL(SDD_EINVAL, "chunk length must be a positive multiple of the largest decimation");
  const int64_t N = chunk_nsamp;
  const int64_t R = ((p->overlap + N - 1) / N + s->d.ring_chunks) * N;
  const int64_t iws = item_workspace(p, N);
  if (iws < 0) return SDD_EINVAL;
  *bytes = R * p->nchan;
  return SDD_OK;
}

extern "C" sdd_status sdd_stream_open(sdd_server* s, const sdd_plan* p, int64_t chunk_nsamp,
                                      uint64_t tag, sdd_stream** out) {
  clear_error();
  if (!s || !p || !out) SDD_FAIL(SDD_EINVAL, "null argument");
  *out = nullptr;
  if (p->layout != SDD_TIME_MAJOR) SDD_FAIL(SDD_EINVAL, "streams take time-major (spectra) plans");
  if (p->device != s->d.device) SDD_FAIL(SDD_EINVAL, "plan and server use different devices");
  if (chunk_nsamp < 1 || chunk_nsamp % p->dec_max != 0)
    SDD_FAIL(SDD_EINVAL, "chunk length must be a positive multiple of the largest decimation");
  const int64_t N = chunk_nsamp;
  const int64_t R = ((p->overlap + N - 1) / N + s->d.ring_chunks) * N;
  const int64_t iws = item_workspace(p, N);
  if (iws < 0) return SDD_EINVAL;
  const int64_t ring_bytes = R * p->nchan;
  const int64_t out_bytes = result_bytes(p, s->d.cap);
  std::unique_lock<std::mutex> lk(s->mu);
  // Admission by footprint: the ring, plus slot growth if this beam's chunks
  // need more workspace or result space than the slots hold. Slots are only
  // resized while idle; waiting for that releases the lock, so every limit is
  // checked again after each wait (another open may have taken the room).
  // Nothing else releases the lock before the ring is counted in hbm_used.
  for (;;) {
    if ((int32_t)s->streams.size() >= s->d.max_beams)
      SDD_FAIL(SDD_EAGAIN, "server holds its maximum of %d beams", s->d.max_beams);
    int64_t grow = 0;
    for (const auto& sl : s->slots) {
      grow += std::max<int64_t>(0, slot_ws_bytes(s, iws) - sl.ws_cap);
      grow += std::max<int64_t>(0, (int64_t)s->d.max_batch * out_bytes - sl.out_cap);
    }
    if (s->hbm_used + ring_bytes + grow > s->d.hbm_budget)
      SDD_FAIL(SDD_EAGAIN, "beam needs %lld bytes; %lld of %lld in use",
               (long long)(ring_bytes + grow), (long long)s->hbm_used,
               (long long)s->d.hbm_budget);
    if (grow == 0) break;
    bool idle = true;
    for (const auto& sl : s->slots) idle = idle && !sl.busy;
    if (!idle) {
      s->cv_done.wait(lk);
      continue;
    }
    sdd_status gs = grow_slots_locked(s, iws, out_bytes);
    if (gs != SDD_OK) return gs;
    break;
  }
  auto st = std::make_unique<sdd_stream>();
  st->srv = s;
  st->plan = p;
  st->tag = tag;
  st->N = N;
  st->O = p->overlap;
  st->R = R;
  st->ring_bytes = ring_bytes;
  st->item_ws = iws;
  if (!fake(s)) {
    DeviceGuard g(s->d.device);
    if (hipMalloc(&st->ring, ring_bytes) != hipSuccess)
      SDD_FAIL(SDD_ENOMEM, "ring allocation of %lld bytes failed", (long long)ring_bytes);
    if (hipStreamCreateWithFlags(&st->copy_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipFree(st->ring);
      SDD_FAIL(SDD_EDEVICE, "stream creation failed");
    }
    sdd_status us = plan_upload(p);
    if (us != SDD_OK) {
      (void)hipFree(st->ring);
      (void)hipStreamDestroy(st->copy_stream);
      return us;
    }
  }
  s->hbm_used += ring_bytes;
  *out = st.get();
  s->streams.push_back(st.release());
  return SDD_OK;
}

extern "C" sdd_status sdd_stream_submit(sdd_stream* st, const uint8_t* chunk, int64_t nsamp,
                                        uint64_t seq, int32_t on_device) {
  clear_error();
  if (!st || (!chunk && !fake(st->srv))) SDD_FAIL(SDD_EINVAL, "null argument");
  sdd_server* s = st->srv;
  if (nsamp != st->N) SDD_FAIL(SDD_EINVAL, "chunk has %lld samples, stream takes %lld",
                               (long long)nsamp, (long long)st->N);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (st->closing) SDD_FAIL(SDD_ESTATE, "stream is closing");
    if ((int64_t)seq != st->submitted)
      SDD_FAIL(SDD_ESTATE, "sequence gap: got chunk %llu, expected %lld",
               (unsigned long long)seq, (long long)st->submitted);
    // rows [sN, (s+1)N) hold samples the oldest unfinished output chunk needs?
    if ((st->submitted + 1) * st->N - st->R > st->oldest_pending * st->N)
      SDD_FAIL(SDD_EAGAIN, "ring full: output chunk %lld still pending", (long long)st->oldest_pending);
  }
  if (!fake(s)) {
    DeviceGuard g(s->d.device);
    uint8_t* dst = st->ring + ((int64_t)seq * st->N % st->R) * st->plan->nchan;
    const int64_t bytes = st->N * st->plan->nchan;
    SDD_HIP_TRY(hipMemcpyAsync(dst, chunk, bytes,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               st->copy_stream));
    SDD_HIP_TRY(hipStreamSynchronize(st->copy_stream));
  }
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted++;
  st->submit_times.emplace_back((int64_t)seq, now_ns());
  while (st->submit_times.size() > 64) st->submit_times.pop_front();
  s->cv_sched.notify_all();
  return SDD_OK;
}

namespace {

// Checkpoint of a stream: this header, then the spectra [count][nchan] of
// samples first_sample .. first_sample + count - 1.
struct SnapHeader {
  uint64_t magic;
  int32_t version, nchan;
  int64_t N, O, submitted, next_out, first_sample, count;
};
constexpr uint64_t kSnapMagic = 0x3150414e53444453ull;  // "SDDSNAP1"

// Copies samples [t0, t0 + n) between host memory and the ring rows they
// occupy (t mod R), in at most two contiguous pieces.
sdd_status ring_copy(sdd_stream* st, int64_t t0, int64_t n, uint8_t* host, bool to_host) {
  const int64_t C = st->plan->nchan;
  int64_t done = 0;
  while (done < n) {
    const int64_t r = (t0 + done) % st->R;
    const int64_t piece = std::min(n - done, st->R - r);
    uint8_t* dev = st->ring + r * C;
    uint8_t* h = host + done * C;
    if (to_host)
      SDD_HIP_TRY(hipMemcpyAsync(h, dev, piece * C, hipMemcpyDeviceToHost, st->copy_stream));
    else
      SDD_HIP_TRY(hipMemcpyAsync(dev, h, piece * C, hipMemcpyHostToDevice, st->copy_stream));
    done += piece;
  }
  SDD_HIP_TRY(hipStreamSynchronize(st->copy_stream));
  return SDD_OK;
}

}  // namespace

extern "C" sdd_status sdd_stream_snapshot(sdd_stream* st, void* host_out, int64_t bytes,
                                          int64_t* needed) {
  clear_error();
  if (!st || !needed) SDD_FAIL(SDD_EINVAL, "null argument");
  sdd_server* s = st->srv;
  std::unique_lock<std::mutex> lk(s->mu);
  if (st->closing) SDD_FAIL(SDD_ESTATE, "stream is closing");
  // the oldest sample an output chunk not yet scheduled needs; output chunks
  // already scheduled finish (and are polled) as usual
  const int64_t first = st->next_out * st->N;
  const int64_t count = std::max<int64_t>(0, st->submitted * st->N - first);
  *needed = (int64_t)sizeof(SnapHeader) + count * st->plan->nchan;
  if (!host_out) return SDD_OK;
  if (bytes < *needed)
    SDD_FAIL(SDD_ENOMEM, "snapshot needs %lld bytes", (long long)*needed);
  st->frozen = true;  // the recorded next output chunk stays unscheduled while we read
  SnapHeader h{};
  h.magic = kSnapMagic;
  h.version = 1;
  h.nchan = st->plan->nchan;
  h.N = st->N;
  h.O = st->O;
  h.submitted = st->submitted;
  h.next_out = st->next_out;
  h.first_sample = first;
  h.count = count;
  lk.unlock();
  // submits of this stream come from its caller, not concurrently with this
  // call, so the ring rows of [first, first + count) are stable
  std::memcpy(host_out, &h, sizeof(h));
  uint8_t* data = static_cast<uint8_t*>(host_out) + sizeof(h);
  sdd_status rc = SDD_OK;
  if (fake(s)) {
    std::memset(data, 0, (size_t)(count * st->plan->nchan));
  } else if (count > 0) {
    DeviceGuard g(s->d.device);
    rc = ring_copy(st, first, count, data, true);
  }
  lk.lock();
  st->frozen = false;
  s->cv_sched.notify_all();
  return rc;
}

extern "C" sdd_status sdd_stream_restore(sdd_server* s, const sdd_plan* p, const void* snapshot,
                                         int64_t bytes, uint64_t tag, sdd_stream** out) {
  clear_error();
  if (!s || !p || !snapshot || !out) SDD_FAIL(SDD_EINVAL, "null argument");
  *out = nullptr;
  SnapHeader h;
  if (bytes < (int64_t)sizeof(h)) SDD_FAIL(SDD_EINVAL, "snapshot shorter than its header");
  std::memcpy(&h, snapshot, sizeof(h));
  if (h.magic != kSnapMagic || h.version != 1) SDD_FAIL(SDD_EINVAL, "not a stream snapshot");
  if (h.nchan != p->nchan || h.O != p->overlap)
    SDD_FAIL(SDD_EINVAL, "snapshot of %d channels and overlap %lld does not fit this plan",
             h.nchan, (long long)h.O);
  if (h.N < 1 || h.submitted < 0 || h.next_out < 0 || h.first_sample != h.next_out * h.N ||
      h.count != std::max<int64_t>(0, h.submitted * h.N - h.first_sample) ||
      bytes < (int64_t)sizeof(h) + h.count * h.nchan)
    SDD_FAIL(SDD_EINVAL, "inconsistent snapshot");
  sdd_stream* st = nullptr;
  sdd_status rc = sdd_stream_open(s, p, h.N, tag, &st);
  if (rc != SDD_OK) return rc;
  if (h.count > st->R) {
    sdd_stream_close(st);
    SDD_FAIL(SDD_EINVAL, "snapshot holds more samples than the ring");
  }
  if (!fake(s) && h.count > 0) {
    DeviceGuard g(s->d.device);
    const uint8_t* data = static_cast<const uint8_t*>(snapshot) + sizeof(h);
    rc = ring_copy(st, h.first_sample, h.count, const_cast<uint8_t*>(data), false);
    if (rc != SDD_OK) {
      sdd_stream_close(st);
      return rc;
    }
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = h.submitted;
    st->next_out = h.next_out;
    st->oldest_pending = h.next_out;
    s->cv_sched.notify_all();
  }
  *out = st;
  return SDD_OK;
}

extern "C" sdd_status sdd_stream_close(sdd_stream* st) {
  clear_error();
  if (!st) return SDD_OK;
  sdd_server* s = st->srv;
  std::unique_lock<std::mutex> lk(s->mu);
  st->closing = true;  // no new submits; unscheduled output chunks are dropped
  s->cv_done.wait(lk, [&] { return st->inflight == 0; });
  s->streams.erase(std::find(s->streams.begin(), s->streams.end(), st));
  s->hbm_used -= st->ring_bytes;
  lk.unlock();
  if (!fake(s)) {
    DeviceGuard g(s->d.device);
    (void)hipFree(st->ring);
    (void)hipStreamDestroy(st->copy_stream);
  }
  delete st;
  return SDD_OK;
}

extern "C" sdd_status sdd_stream_poll(sdd_server* s, sdd_result* out, int32_t max,
                                      int32_t timeout_us, int32_t* n_out) {
  clear_error();
  if (!s || !n_out || max < 0 || (max > 0 && !out)) SDD_FAIL(SDD_EINVAL, "bad argument");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->results.empty() && timeout_us > 0)
    s->cv_poll.wait_for(lk, std::chrono::microseconds(timeout_us),
                        [&] { return !s->results.empty() || s->stop; });
  else if (s->results.empty() && timeout_us < 0)
    s->cv_poll.wait(lk, [&] { return !s->results.empty() || s->stop; });
  int32_t n = 0;
  while (n < max && !s->results.empty()) {
    ResultBox* b = s->results.front();
    s->results.pop_front();
    s->out_results[b] = b;
    out[n++] = b->r;
  }
  *n_out = n;
  if (n == 0) SDD_FAIL(SDD_ETIMEDOUT, "no result within %d us", timeout_us);
  return SDD_OK;
}

extern "C" sdd_status sdd_result_release(sdd_server* s, sdd_result* r) {
  clear_error();
  if (!s || !r || !r->handle) SDD_FAIL(SDD_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->out_results.find(r->handle);
  if (it == s->out_results.end()) SDD_FAIL(SDD_EINVAL, "unknown or released result");
  ResultBox* b = it->second;
  s->out_results.erase(it);
  r->handle = nullptr;
  free_box(s, b);
  return SDD_OK;
}

extern "C" sdd_status sdd_stream_keep_planes(sdd_stream* st, int32_t on) {
  clear_error();
  if (!st) SDD_FAIL(SDD_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(st->srv->mu);
  st->keep_planes = on != 0;
  return SDD_OK;
}

extern "C" sdd_status sdd_result_copy_planes(sdd_server* s, const sdd_result* r,
                                             uint32_t* const* d_dst, const int64_t* dst_pitch,
                                             void* stream) {
  clear_error();
  if (!s || !r || !r->handle || !d_dst || !dst_pitch) SDD_FAIL(SDD_EINVAL, "null argument");
  const ResultBox* b = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->out_results.find(r->handle);
    if (it == s->out_results.end()) SDD_FAIL(SDD_EINVAL, "unknown or released result");
    b = it->second;
  }
  const sdd_result& br = b->r;
  if (br.nplanes < 1) SDD_FAIL(SDD_EINVAL, "the result holds no planes");
  for (int q = 0; q < br.nplanes; ++q)
    if (!d_dst[q] || dst_pitch[q] < br.plane_cols[q])
      SDD_FAIL(SDD_EINVAL, "range %d: destination pitch %lld < %lld columns", q,
               (long long)dst_pitch[q], (long long)br.plane_cols[q]);
  DeviceGuard g(s->d.device);
  for (int q = 0; q < br.nplanes; ++q)
    SDD_HIP_TRY(hipMemcpy2DAsync(d_dst[q], (size_t)dst_pitch[q] * 4, br.d_planes[q],
                                 (size_t)br.plane_pitch[q] * 4, (size_t)br.plane_cols[q] * 4,
                                 (size_t)br.plane_rows[q], hipMemcpyDeviceToDevice,
                                 static_cast<hipStream_t>(stream)));
  return SDD_OK;
}

extern "C" sdd_status sdd_server_query(sdd_server* s, sdd_server_stats* out) {
  clear_error();
  if (!s || !out) SDD_FAIL(SDD_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->open_streams = (int32_t)s->streams.size();
  out->hbm_used = s->hbm_used;
  out->batches = s->batches;
  out->chunks = s->chunks;
  out->busy_ms = s->busy_ms;
  out->queued_results = (int32_t)s->results.size();
  return SDD_OK;
}

extern "C" sdd_status sdd_server_destroy(sdd_server* s) {
  clear_error();
  if (!s) return SDD_OK;
  std::vector<sdd_stream*> open;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    open = s->streams;
  }
  for (sdd_stream* st : open) sdd_stream_close(st);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
    s->cv_poll.notify_all();
  }
  s->th_sched.join();
  s->th_done.join();
  for (ResultBox* b : s->results) free_box(s, b);
  for (auto& kv : s->out_results) free_box(s, kv.second);
  if (!fake(s)) {
    DeviceGuard g(s->d.device);
    for (auto& sl : s->slots) {
      if (sl.ws) (void)hipFree(sl.ws);
      if (sl.dout) (void)hipFree(sl.dout);
      if (sl.hout) (void)hipHostFree(sl.hout);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
  }
  delete s;
  return SDD_OK;
}
