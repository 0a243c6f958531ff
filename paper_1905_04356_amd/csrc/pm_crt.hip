// pm_crt.hip -- single-product Chinese remaindering kernel (device work in
// pm_crt_dev.h) and the opt-in residue check.
#include "pm_crt_dev.h"
#include "pm_profile.h"

namespace pm {

template <typename TOut>
__global__ __launch_bounds__(256) void crt_kernel(CrtLaunch a) {
  crt_range<TOut>(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, a.count,
                  (uint64_t)gridDim.x * blockDim.x);
}

int launch_crt(const CrtLaunch& a, int out_elem_bytes, hipStream_t s) {
  uint64_t blocks = (a.count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  if (out_elem_bytes == 8)
    return launch(crt_kernel<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    return launch(crt_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, a);
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
    return launch(check_residues_kernel<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s, p,
                  (const uint64_t*)x, count, counter);
  else
    return launch(check_residues_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, p,
                  (const uint32_t*)x, count, counter);
}

// Coefficients of A B from A B mod (x^L - 1): rows L .. L + t - 1 of C hold
// the true top coefficients, which wrapped onto rows 0 .. t - 1; subtract
// them there (count = t m k elements, off = L m k).
template <typename T>
__global__ __launch_bounds__(256) void unwrap_kernel(T* C, uint64_t count, uint64_t off,
                                                     uint64_t p) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const T a = C[i], b = C[off + i];
    C[i] = a >= b ? a - b : (T)(a + (p - b));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void neg_mod_kernel(const T* X, T* Y, uint64_t count,
                                                      uint64_t p) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const T x = X[i];
    Y[i] = x ? (T)(p - x) : (T)0;
  }
}

int launch_neg_mod(uint64_t p, const void* X, void* Y, uint64_t count, int elem_bytes,
                   hipStream_t s) {
  uint64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) return hipSuccess;
  if (elem_bytes == 8)
    return launch(neg_mod_kernel<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                  (const uint64_t*)X, (uint64_t*)Y, count, p);
  else
    return launch(neg_mod_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                  (const uint32_t*)X, (uint32_t*)Y, count, p);
}

int launch_unwrap(void* C, uint64_t count, uint64_t off, uint64_t p, int elem_bytes,
                  hipStream_t s) {
  uint64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) return hipSuccess;
  if (elem_bytes == 8)
    return launch(unwrap_kernel<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                  (uint64_t*)C, count, off, p);
  else
    return launch(unwrap_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                  (uint32_t*)C, count, off, p);
}

}  // namespace pm
