// pm_profile.h -- RAII event pair around one kernel launch (when profiling).
#pragma once
#include <hip/hip_runtime.h>

namespace pm {

enum KernelKind {
  K_NTT_FWD = 0, K_POINTWISE = 1, K_NTT_INV = 2, K_CRT = 3, K_BATCHED = 4,
  K_VDM_EVAL = 5, K_VDM_INTERP = 6
};

bool profiling();

class KernelTimer {
 public:
  KernelTimer(int kind, hipStream_t s);
  ~KernelTimer();
  KernelTimer(const KernelTimer&) = delete;
  KernelTimer& operator=(const KernelTimer&) = delete;

 private:
  int kind_;
  hipStream_t s_;
  hipEvent_t a_{}, b_{};
  bool armed_ = false;
};

}  // namespace pm
