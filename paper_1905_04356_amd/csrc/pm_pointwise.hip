// pm_pointwise.hip -- single-product pointwise kernels and launchers (the
// per-workgroup work is in pm_pointwise_dev.h).
#include "pm_pointwise_dev.h"
#include "pm_profile.h"

#include <stdlib.h>

namespace pm {

template <bool STAGED>
__global__ __launch_bounds__(256) void pointwise_valu_kernel(PointwiseLaunch a) {
  extern __shared__ uint32_t sm[];
  pointwise_valu_tile<STAGED>(a, blockIdx.x, blockIdx.y, sm);
}

template <int NT>
__global__ __launch_bounds__(NT) void pointwise_mfma_kernel(PointwiseLaunch a) {
  extern __shared__ uint32_t smem[];
  pointwise_mfma_tile(a, blockIdx.x, blockIdx.y, smem);
}

int launch_pointwise(const PointwiseLaunch& a, int nprimes, hipStream_t s) {
  const size_t lds = sizeof(uint32_t) * ((size_t)a.m * a.n + (size_t)a.n * a.k);
  if (lds > 128 * 1024) {
    // operands too large to stage: read them from global memory (L2)
    return launch(pointwise_valu_kernel<false>, dim3(a.L, nprimes), dim3(256), 0, s, a);
  }
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)pointwise_valu_kernel<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return launch(pointwise_valu_kernel<true>, dim3(a.L, nprimes), dim3(256), lds, s, a);
}


size_t pointwise_mfma_lds(int m, int n, int k) {
  const size_t mp = (m + 15) & ~15, kp = (k + 15) & ~15, np = (n + 63) & ~63;
  return 4 * (mp + kp) * (np + 16);
}

// Up to 44 KiB of limb planes: 256 threads, so that several workgroups share
// a CU.  Above it, 512 threads: each thread stages half as many items and
// so waits for fewer load round trips (measured on single products: 128x64x8
// 44 -> 40 us, 64x128x32 70 -> 53 us, 128x32x64 109 -> 78 us, while 41 KiB
// and below lose).  Tuning knob PM_TUNE_PW_SMALL_LDS (bytes).
size_t pointwise_small_lds() {
  static const size_t v = [] {
    const char* e = getenv("PM_TUNE_PW_SMALL_LDS");
    return e && *e ? (size_t)strtoull(e, nullptr, 10) : (size_t)44 * 1024;
  }();
  return v;
}

int launch_pointwise_mfma(const PointwiseLaunch& a, int nprimes, hipStream_t s) {
  const size_t lds = pointwise_mfma_lds(a.m, a.n, a.k);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds <= pointwise_small_lds()) {
    return launch(pointwise_mfma_kernel<256>, dim3(a.L, nprimes), dim3(256), lds, s, a);
  }
  hipError_t e = hipFuncSetAttribute((const void*)pointwise_mfma_kernel<512>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return launch(pointwise_mfma_kernel<512>, dim3(a.L, nprimes), dim3(512), lds, s, a);
}

}  // namespace pm
