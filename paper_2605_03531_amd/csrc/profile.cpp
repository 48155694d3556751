// Optional per-stage kernel timing with HIP events (benchmark support).
#include <mutex>
#include <vector>

#include "sdd_internal.h"

namespace sdd {
namespace {
struct Pending {
  int stage;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
double g_ms[SDD_NSTAGES] = {0};
int64_t g_n[SDD_NSTAGES] = {0};

void drain_locked() {
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_ms[p.stage] += ms;
      g_n[p.stage] += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
}
}  // namespace

StageTimer::StageTimer(int stage, hipStream_t s) : stage_(stage), s_(s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (hipEventCreate(&a_) != hipSuccess) return;
  if (hipEventCreate(&b_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    return;
  }
  if (hipEventRecord(a_, s_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    (void)hipEventDestroy(b_);
    return;
  }
  active_ = true;
}

StageTimer::~StageTimer() {
  if (!active_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipEventRecord(b_, s_) == hipSuccess) {
    g_pending.push_back({stage_, a_, b_});
  } else {
    (void)hipEventDestroy(a_);
    (void)hipEventDestroy(b_);
  }
}

}  // namespace sdd

using namespace sdd;

extern "C" sdd_status sdd_profile_enable(int32_t on) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  if (on) {
    drain_locked();
    for (int k = 0; k < SDD_NSTAGES; ++k) {
      g_ms[k] = 0.0;
      g_n[k] = 0;
    }
  }
  g_on = on != 0;
  return SDD_OK;
}

extern "C" sdd_status sdd_profile_read(int32_t stage, double* total_ms, int64_t* launches) {
  clear_error();
  if (stage < 0 || stage >= SDD_NSTAGES || !total_ms || !launches)
    SDD_FAIL(SDD_EINVAL, "bad stage or null output");
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  *total_ms = g_ms[stage];
  *launches = g_n[stage];
  return SDD_OK;
}
