// pm_pointwise.hip -- single-product pointwise kernels and launchers (the
// per-workgroup work is in pm_pointwise_dev.h).
#include "pm_pointwise_dev.h"
#include "pm_profile.h"

#include <stdlib.h>

#include <algorithm>

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

template <int NT, int PA, int PB>
__global__ __launch_bounds__(NT) void pointwise_mfma_pipe_kernel(PointwiseLaunch a) {
  extern __shared__ uint32_t smem[];
  pointwise_mfma_pipe_any<NT, PA, PB>(a, blockIdx.y, blockIdx.x, a.L, gridDim.x, smem);
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
  if (n <= 16) return 4 * (mp + kp) * kK16Row + kK16Row;  // packed contraction
  return 4 * (mp + kp) * (np + 16);
}

// Pipelined-kernel variant for a shape with 512 threads: 1 (4 A groups and
// one B block per thread: 122 VGPRs, two workgroups per CU), 2 (8 and 2:
// 154 VGPRs, one), or 0 when the shape needs more registers, k is not a
// multiple of 4 or n <= 16 (packed contraction).  knob 0 never pipelines,
// 1 or 2 forces that variant where it suffices.
int pointwise_pipe_variant(int m, int n, int k, int knob) {
  if (knob == 0 || k % 4 != 0 || n <= 16) return 0;  // n <= 16: packed contraction
  const long mp = (m + 15) & ~15, kp = (k + 15) & ~15, ng = ((n + 63) & ~63) >> 2;
  const long need_a = (mp * ng + 511) / 512, need_b = (ng * (kp / 4) + 511) / 512;
  const bool small = need_a <= 4 && need_b <= 1, big = need_a <= 8 && need_b <= 2;
  if (knob == 1) return small ? 1 : 0;
  if (knob == 2) return big ? 2 : 0;
  return small ? 1 : big ? 2 : 0;
}

namespace {
int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

// One resident workgroup per slot of the chip, each running every
// gridDim.x-th point.
template <int PA, int PB>
int launch_pipe(const PointwiseLaunch& a, int nprimes, size_t lds, hipStream_t s) {
  const void* fn = (const void*)pointwise_mfma_pipe_kernel<512, PA, PB>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 512, lds);
  if (e != hipSuccess) return e;
  const int cus = cu_count();
  if (per_cu < 1 || cus < 1) return hipErrorInvalidValue;
  const long g = std::min<long>(a.L, (long)per_cu * cus);
  return launch(pointwise_mfma_pipe_kernel<512, PA, PB>, dim3((unsigned)g, nprimes), dim3(512),
                lds, s, a);
}
}  // namespace

int launch_pointwise_mfma(const PointwiseLaunch& a, int nprimes, hipStream_t s) {
  const size_t lds = pointwise_mfma_lds(a.m, a.n, a.k);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  // small limb planes: 256 threads, so that several workgroups share a CU;
  // larger ones: 512 threads, each waiting for fewer load round trips
  if (lds <= (size_t)a.small_lds) {
    return launch(pointwise_mfma_kernel<256>, dim3(a.L, nprimes), dim3(256), lds, s, a);
  }
  switch (pointwise_pipe_variant(a.m, a.n, a.k, a.pipe)) {
    case 1: return launch_pipe<4, 1>(a, nprimes, lds, s);
    case 2: return launch_pipe<8, 2>(a, nprimes, lds, s);
    default: break;
  }
  hipError_t e = hipFuncSetAttribute((const void*)pointwise_mfma_kernel<512>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return launch(pointwise_mfma_kernel<512>, dim3(a.L, nprimes), dim3(512), lds, s, a);
}

}  // namespace pm
