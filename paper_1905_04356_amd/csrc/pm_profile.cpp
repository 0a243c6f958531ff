// pm_profile.cpp -- optional per-kernel device timing with HIP events.
#include "pm_profile.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/pm.h"

namespace pm {

namespace {
struct Rec {
  int kind;
  hipEvent_t a, b;
};
std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Rec> g_recs;
bool g_failed = false;
}  // namespace

bool profiling() { return g_on.load(std::memory_order_relaxed) != 0; }

KernelTimer::KernelTimer(int kind, hipStream_t s) : kind_(kind), s_(s) {
  if (!profiling()) return;
  // no timing inside a stream capture: the events would become graph nodes
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
    std::lock_guard<std::mutex> l(g_mu);
    g_failed = true;
    return;
  }
  if (hipEventRecord(a_, s_) != hipSuccess) {
    std::lock_guard<std::mutex> l(g_mu);
    g_failed = true;
    return;
  }
  armed_ = true;
}

KernelTimer::~KernelTimer() {
  if (!armed_) return;
  std::lock_guard<std::mutex> l(g_mu);
  if (hipEventRecord(b_, s_) != hipSuccess) {
    g_failed = true;
    return;
  }
  g_recs.push_back(Rec{kind_, a_, b_});
}

}  // namespace pm

extern "C" {

pm_status pm_profile_begin(void) {
  std::lock_guard<std::mutex> l(pm::g_mu);
  pm::g_recs.clear();
  pm::g_failed = false;
  pm::g_on.store(1);
  return PM_OK;
}

pm_status pm_profile_end(pm_kernel_stats* out) {
  if (!out) return PM_EINVAL;
  pm::g_on.store(0);
  std::lock_guard<std::mutex> l(pm::g_mu);
  memset(out, 0, sizeof *out);
  bool bad = pm::g_failed;
  for (auto& r : pm::g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      bad = true;
    if (r.kind >= 0 && r.kind < PM_KERNEL_KINDS) {
      out->total_ms[r.kind] += ms;
      out->launches[r.kind] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  pm::g_recs.clear();
  return bad ? PM_EDEVICE : PM_OK;
}

}  // extern "C"
