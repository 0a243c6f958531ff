// pm_probe.hip -- a measurement of the VALU rate that bounds the transforms.
//
// The butterflies are built from 32-bit multiplies (the high and low halves
// of Shoup's products), adds and minimums; the ALU roofline counts every
// VALU instruction as one lane-op at the chip's issue rate (256 CUs x 4
// SIMDs x 16 lanes x 2.4 GHz).  This kernel checks that 32-bit high
// multiplies issue at that rate: each thread runs kChains independent
// chains x <- mulhi(x, m), so no instruction waits for the previous one
// of its chain, and the caller times the launch.
#include "pm_kernels.h"
#include "pm_profile.h"

namespace pm {

namespace {

constexpr int kProbeChains = 8;

__global__ __launch_bounds__(256) void probe_mulhi_kernel(uint32_t* out, uint32_t iters,
                                                          uint32_t m) {
  uint32_t x[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) x[c] = threadIdx.x + 0x9E3779B9u * (c + 1);
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) x[c] = __umulhi(x[c], m);
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) acc ^= x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

int launch_probe_mulhi(uint32_t* out, uint32_t blocks, uint32_t iters, uint32_t m,
                       hipStream_t s) {
  return launch(probe_mulhi_kernel, dim3(blocks), dim3(256), 0, s, out, iters, m);
}

}  // namespace pm
