// pm_pointwise.hip -- the matrix products at the evaluation points.
//
// After evaluation, the polynomial-matrix product becomes L independent
// products of an m x n by an n x k matrix over F_q, one per point
// (Hyun, Neiger, Schost, ISSAC 2019, Section 2, "Polynomial matrix
// multiplication": the n^omega d term of the evaluation/interpolation
// bound; plain cubic products per point, Section 2, "Matrix
// multiplication").  The factor L^{-1} of the inverse transform is applied
// here, once per output value.
//
// VALU variant: one workgroup per point; the two matrices are staged in LDS,
// each thread accumulates full 64-bit products in a 96-bit sum (64-bit low
// word plus carry count) and reduces once per output.
#include "pm_arith.h"
#include "pm_kernels.h"

namespace pm {

template <bool STAGED>
__global__ __launch_bounds__(256) void pointwise_valu_kernel(PointwiseLaunch a) {
  extern __shared__ uint32_t sm[];
  const int t = blockIdx.x;
  const int prime = blockIdx.y;
  const PrimeConst& P = a.pc[prime];
  const uint32_t q = P.q;
  const size_t mn = (size_t)a.m * a.n, nk = (size_t)a.n * a.k, mk = (size_t)a.m * a.k;
  const uint32_t* A = a.ahat + a.prime_stride * prime + (size_t)t * mn;
  const uint32_t* B = a.bhat + a.prime_stride * prime + (size_t)t * nk;
  uint32_t* C = a.chat + a.prime_stride * prime + (size_t)t * mk;
  const uint32_t* sa = A;
  const uint32_t* sb = B;
  if (STAGED) {
    for (size_t i = threadIdx.x; i < mn; i += blockDim.x) sm[i] = A[i];
    for (size_t i = threadIdx.x; i < nk; i += blockDim.x) sm[mn + i] = B[i];
    __syncthreads();
    sa = sm;
    sb = sm + mn;
  }
  // 2^64 mod q, to fold the carry count back in.
  const uint64_t r64 = ((~0ull) % q + 1) % q;
  for (size_t o = threadIdx.x; o < mk; o += blockDim.x) {
    const int i = (int)(o / a.k), j = (int)(o % a.k);
    uint64_t lo = 0;
    uint32_t hi = 0;
    for (int l = 0; l < a.n; ++l) {
      const uint64_t prod = (uint64_t)sa[(size_t)i * a.n + l] * sb[(size_t)l * a.k + j];
      lo += prod;
      hi += lo < prod;
    }
    const uint32_t v = reduce_u64((uint64_t)hi * r64 + reduce_u64(lo, q, P.mu), q, P.mu);
    C[o] = mul_shoup(v, P.linv, P.linv_p, q);
  }
}

int launch_pointwise(const PointwiseLaunch& a, int nprimes, hipStream_t s) {
  const size_t lds = sizeof(uint32_t) * ((size_t)a.m * a.n + (size_t)a.n * a.k);
  if (lds > 128 * 1024) {
    // operands too large to stage: read them from global memory (L2)
    hipLaunchKernelGGL(pointwise_valu_kernel<false>, dim3(a.L, nprimes), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)pointwise_valu_kernel<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(pointwise_valu_kernel<true>, dim3(a.L, nprimes), dim3(256), lds, s, a);
  return hipGetLastError();
}

}  // namespace pm
