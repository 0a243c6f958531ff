// pm_profile.cpp -- optional per-kernel device timing with HIP events.
#include "pm_profile.h"

#include <hip/hip_ext.h>
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
  int dev;
  hipEvent_t a, b;
};

int current_device() {
  int dev = 0;
  return hipGetDevice(&dev) == hipSuccess ? dev : 0;
}
std::atomic<int> g_on{0};  // 0 off, 1 timing, 2 paused
std::mutex g_mu;
std::vector<Rec> g_recs;
bool g_failed = false;
thread_local int t_kind = -1;  // kind of the innermost per-launch scope

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// Events of finished timing sessions, per device, for the next timed
// launches (creating two events per launch costs more host time than the
// launch itself for small products).
std::vector<std::vector<hipEvent_t>> g_pool;

// timing-only events: without the system-scope fence, completing one does
// not write back and invalidate the caches
bool make_pair(hipEvent_t* a, hipEvent_t* b) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  {
    std::lock_guard<std::mutex> l(g_mu);
    if ((int)g_pool.size() > dev && g_pool[dev].size() >= 2) {
      *a = g_pool[dev].back();
      g_pool[dev].pop_back();
      *b = g_pool[dev].back();
      g_pool[dev].pop_back();
      return true;
    }
  }
  if (hipEventCreateWithFlags(a, hipEventDisableSystemFence) != hipSuccess) return false;
  if (hipEventCreateWithFlags(b, hipEventDisableSystemFence) != hipSuccess) {
    (void)hipEventDestroy(*a);
    return false;
  }
  return true;
}

void failed() {
  std::lock_guard<std::mutex> l(g_mu);
  g_failed = true;
}
}  // namespace

bool profiling() { return g_on.load(std::memory_order_relaxed) == 1; }

KernelTimer::KernelTimer(int kind, hipStream_t s, bool scope_events)
    : kind_(kind), prev_kind_(t_kind), s_(s) {
  t_kind = scope_events ? -1 : kind;
  if (!scope_events || !profiling() || capturing(s_)) return;
  if (!make_pair(&a_, &b_)) {
    failed();
    return;
  }
  if (hipEventRecord(a_, s_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    (void)hipEventDestroy(b_);
    failed();
    return;
  }
  armed_ = true;
}

KernelTimer::~KernelTimer() {
  t_kind = prev_kind_;
  if (!armed_) return;
  std::lock_guard<std::mutex> l(g_mu);
  if (hipEventRecord(b_, s_) != hipSuccess) {
    g_failed = true;
    return;
  }
  g_recs.push_back(Rec{kind_, current_device(), a_, b_});
}

hipError_t launch_kernel(const void* fn, dim3 grid, dim3 block, void** args, size_t lds,
                         hipStream_t s) {
  hipError_t e;
  hipEvent_t a, b;
  bool timed = t_kind >= 0 && profiling() && !capturing(s);
  if (timed && !make_pair(&a, &b)) {
    failed();
    timed = false;
  }
  if (timed) {
    e = hipExtLaunchKernel(fn, grid, block, args, lds, s, a, b, 0);
    if (e == hipSuccess) {
      std::lock_guard<std::mutex> l(g_mu);
      g_recs.push_back(Rec{t_kind, current_device(), a, b});
    } else {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } else {
    e = hipLaunchKernel(fn, grid, block, args, lds, s);
  }
  const hipError_t last = hipGetLastError();
  return e != hipSuccess ? e : last;
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

pm_status pm_profile_pause(int32_t paused) {
  std::lock_guard<std::mutex> l(pm::g_mu);
  if (pm::g_on.load() == 0) return PM_EINVAL;
  pm::g_on.store(paused ? 2 : 1);
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
    if (r.dev >= (int)pm::g_pool.size()) pm::g_pool.resize(r.dev + 1);
    pm::g_pool[r.dev].push_back(r.b);
    pm::g_pool[r.dev].push_back(r.a);
  }
  pm::g_recs.clear();
  return bad ? PM_EDEVICE : PM_OK;
}

}  // extern "C"
