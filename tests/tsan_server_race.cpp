// Host-side race check of the streaming server: built with ThreadSanitizer
// on the host code only and run with a server in fake mode (no device memory,
// batches sleep), so the scheduler, completion and caller threads interleave
// for real. Several threads submit to their own beams (retrying on ring-full
// backpressure), one polls and releases results, one queries the server, and
// one beam is checkpointed mid-stream, closed and restored. The program
// checks that every output chunk of every beam arrives exactly once.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <mutex>
#include <set>
#include <thread>
#include <utility>
#include <vector>

#include "spotdd.h"

#define CHECK(x)                                                                 \
  do {                                                                           \
    const sdd_status rc_ = (x);                                                  \
    if (rc_ != SDD_OK) {                                                         \
      std::fprintf(stderr, "%s failed: %d %s\n", #x, (int)rc_, sdd_last_error()); \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

int main() {
  constexpr int kChan = 64, kDm = 16, kBeams = 8, kChunks = 12, kThreadsSubmit = 4;
  constexpr int64_t kN = 1024;
  std::vector<double> f(kChan), dms(kDm);
  for (int c = 0; c < kChan; ++c) f[c] = 750.0 - 200.0 * c / (kChan - 1);
  for (int i = 0; i < kDm; ++i) dms[i] = 50.0 * i / (kDm - 1);
  const int32_t widths[3] = {1, 2, 4};
  sdd_plan_desc pd{};
  pd.freqs_mhz = f.data();
  pd.dm_list = dms.data();
  pd.widths = widths;
  pd.t_samp_s = 81.92e-6;
  pd.nchan = kChan;
  pd.ndm = kDm;
  pd.nwidths = 3;
  pd.threshold = 7.0f;
  pd.layout = SDD_TIME_MAJOR;
  sdd_plan* plan = nullptr;
  CHECK(sdd_plan_create(&pd, &plan));
  sdd_plan_info info{};
  CHECK(sdd_plan_query(plan, &info));

  sdd_server_desc sd{};
  sd.hbm_budget = (int64_t)1 << 40;
  sd.max_beams = 64;
  sd.nstreams = 3;
  sd.max_batch = 4;
  sd.ring_chunks = 2;
  sd.cap = 256;
  sd.batch_flags = SDD_BATCH_PER_ITEM;
  sd.flags = SDD_SERVER_FAKE;
  sd.fake_exec_us = 200;
  sdd_server* srv = nullptr;
  CHECK(sdd_server_create(&sd, &srv));

  std::vector<sdd_stream*> beams(kBeams, nullptr);
  for (int b = 0; b < kBeams; ++b) CHECK(sdd_stream_open(srv, plan, kN, (uint64_t)b, &beams[b]));
  const int64_t per_beam = (kChunks * kN - info.overlap) / kN;
  const int64_t want = per_beam * kBeams;

  std::mutex seen_mu;
  std::set<std::pair<uint64_t, int64_t>> seen;
  std::atomic<int64_t> got{0};
  std::atomic<bool> dup{false}, bad{false}, done_submit{false}, stop{false};

  std::thread poller([&] {
    sdd_result res[16];
    while (got.load() < want && !stop.load()) {
      int32_t n = 0;
      const sdd_status rc = sdd_stream_poll(srv, res, 16, 2000, &n);
      if (rc == SDD_ETIMEDOUT) continue;  // nothing finished within 2 ms
      if (rc != SDD_OK) {
        bad = true;
        return;
      }
      for (int32_t q = 0; q < n; ++q) {
        // a restored beam keeps its tag: (tag, chunk) identifies the output
        {
          std::lock_guard<std::mutex> lk(seen_mu);
          if (!seen.insert({res[q].tag, res[q].chunk}).second) dup = true;
        }
        if (res[q].status != SDD_OK || sdd_result_release(srv, &res[q]) != SDD_OK) bad = true;
      }
      got += n;
    }
  });
  std::thread watcher([&] {
    sdd_server_stats st{};
    while (!done_submit.load()) {
      if (sdd_server_query(srv, &st) != SDD_OK) bad = true;
      std::this_thread::sleep_for(std::chrono::microseconds(300));
    }
  });
  std::vector<std::thread> submitters;
  for (int t = 0; t < kThreadsSubmit; ++t)
    submitters.emplace_back([&, t] {
      for (int64_t k = 0; k < kChunks; ++k)
        for (int b = t; b < kBeams; b += kThreadsSubmit) {
          if (b == 0 && k == kChunks / 2) {
            // checkpoint beam 0, close it, restore it under the same tag
            int64_t need = 0;
            if (sdd_stream_snapshot(beams[0], nullptr, 0, &need) != SDD_OK) bad = true;
            std::vector<unsigned char> snap((size_t)need);
            if (sdd_stream_snapshot(beams[0], snap.data(), need, &need) != SDD_OK) bad = true;
            if (sdd_stream_close(beams[0]) != SDD_OK) bad = true;
            if (sdd_stream_restore(srv, plan, snap.data(), need, 0, &beams[0]) != SDD_OK)
              bad = true;
          }
          sdd_status rc;
          while ((rc = sdd_stream_submit(beams[b], nullptr, kN, (uint64_t)k, 0)) == SDD_EAGAIN)
            std::this_thread::sleep_for(std::chrono::microseconds(100));
          if (rc != SDD_OK) bad = true;
        }
    });
  for (auto& th : submitters) th.join();
  done_submit = true;
  watcher.join();
  const auto t0 = std::chrono::steady_clock::now();
  while (got.load() < want && !bad.load() &&
         std::chrono::steady_clock::now() - t0 < std::chrono::seconds(30))
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  if (got.load() < want) bad = true;
  stop = true;
  poller.join();
  if (bad.load()) {
    std::fprintf(stderr, "failed: %lld of %lld results\n", (long long)got.load(), (long long)want);
    return 1;
  }
  for (auto* b : beams) CHECK(sdd_stream_close(b));
  CHECK(sdd_server_destroy(srv));
  CHECK(sdd_plan_destroy(plan));
  if (dup.load()) {
    std::fprintf(stderr, "an output chunk arrived twice\n");
    return 1;
  }
  std::printf("ok: %lld results from %d beams, each output chunk once\n", (long long)want, kBeams);
  return 0;
}
