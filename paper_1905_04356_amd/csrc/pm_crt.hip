// pm_crt.hip -- Chinese remaindering for moduli that are not FFT primes, and
// the opt-in residue check.
//
// For a modulus p without large 2-power roots of unity, the product is lifted
// to Z[x] (inputs taken in [0, p)), computed modulo r FFT primes whose
// product exceeds every integer coefficient n*d*(p-1)^2, and rebuilt
// (Hyun, Neiger, Schost, ISSAC 2019, Section 2, "Polynomial multiplication":
// 3-primes FFT for primes without Fourier transforms; "Polynomial matrix
// multiplication": lifting F_p[x] to Z[x] modulo a few FFT primes).
//
// Reconstruction is Garner's mixed-radix form: with residues v_i = X mod q_i,
//   y_0 = v_0,  y_i = (...((v_i - y_0) q_0^{-1} - y_1) q_1^{-1} ... - y_{i-1}) q_{i-1}^{-1} mod q_i,
// then X = y_0 + y_1 q_0 + y_2 q_0 q_1 + ... exactly (0 <= X < prod q_i), so
// X mod p = sum_i y_i (prod_{j<i} q_j mod p) mod p.
#include "pm_arith.h"
#include "pm_kernels.h"

namespace pm {

template <typename TOut>
__global__ __launch_bounds__(256) void crt_kernel(CrtLaunch a) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.count;
       idx += stride) {
    uint32_t y[kMaxPrimes];
    for (int i = 0; i < a.r; ++i) {
      const uint32_t qi = a.q[i];
      uint32_t t = a.cq[a.prime_stride * i + idx];
      for (int j = 0; j < i; ++j) {
        const uint32_t yj = reduce_u64(y[j], qi, a.mu[i]);
        t = sub_mod(t, yj, qi);
        t = mul_shoup(t, a.inv[i][j], a.inv_p[i][j], qi);
      }
      y[i] = t;
    }
    uint64_t acc = 0;
    if (a.p <= 0xFFFFFFFFull) {
      for (int i = 0; i < a.r; ++i) acc = (acc + (uint64_t)y[i] * a.radix_mod_p[i] % a.p) % a.p;
    } else {
      for (int i = 0; i < a.r; ++i) {
        acc += mulmod_u64_small(y[i], a.radix_mod_p[i], a.p, a.pinv);
        if (acc >= a.p) acc -= a.p;
      }
    }
    ((TOut*)a.out)[idx] = (TOut)acc;
  }
}

int launch_crt(const CrtLaunch& a, int out_elem_bytes, hipStream_t s) {
  uint64_t blocks = (a.count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  if (out_elem_bytes == 8)
    hipLaunchKernelGGL(crt_kernel<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(crt_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void check_residues_kernel(uint64_t p, const T* x,
                                                             uint64_t count,
                                                             unsigned long long* counter) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long bad = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    bad += (uint64_t)x[i] >= p;
  if (bad) atomicAdd(counter, bad);
}

int launch_check_residues(uint64_t p, const void* x, uint64_t count, int elem_bytes,
                          unsigned long long* counter, hipStream_t s) {
  uint64_t blocks = (count + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks == 0) blocks = 1;
  if (elem_bytes == 8)
    hipLaunchKernelGGL(check_residues_kernel<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                       p, (const uint64_t*)x, count, counter);
  else
    hipLaunchKernelGGL(check_residues_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                       p, (const uint32_t*)x, count, counter);
  return hipGetLastError();
}

}  // namespace pm
