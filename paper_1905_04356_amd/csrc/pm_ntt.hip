// pm_ntt.hip -- batched number-theoretic transforms along the degree axis.
//
// Evaluation at the L-th roots of unity of an FFT prime q and interpolation
// back (Hyun, Neiger, Schost, ISSAC 2019, Section 2, "Polynomial
// multiplication" (FFT paragraph) and "Polynomial matrix multiplication"
// (evaluation/interpolation at roots of unity for FFT primes)).
//
// One workgroup transforms 2^eb_log polynomials held in LDS (L <= 2^15).
// Stages are grouped in passes of up to five radix-2 stages: each thread
// loads 2^r values at stride S from LDS into registers, runs r butterfly
// stages there, and writes them back.  Multiplication by a root of unity uses
// Shoup's precomputed quotient (pm_arith.h); the twiddles of a pass are read
// from a table laid out per thread index j, so a thread reads 2^r - 1
// consecutive pairs.  Residues stay canonical ([0, q)) between stages,
// because 2q < 2^32 but 4q may not be (q can exceed 2^30).
//
// Forward = decimation in frequency on natural-order input: position t of the
// output holds the value at w^bitrev(t).  Inverse = decimation in time on that
// order with w^-1, giving L times the natural-order coefficients.
#include "pm_arith.h"
#include "pm_kernels.h"

namespace pm {

__device__ __forceinline__ int lds_pos(int pos) { return pos + (pos >> 5); }

// One decimation-in-frequency pass of r stages at stride 2^s.
template <int r>
__device__ __forceinline__ void dif_pass(uint32_t* lds, int lds_stride, int logL, int s,
                                         const Tw* __restrict__ tw, int eb_log, uint32_t q) {
  constexpr int R = 1 << r;
  const int S = 1 << s;
  const int per_entry_log = logL - r;
  const int items = 1 << (per_entry_log + eb_log);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int e = it >> per_entry_log;
    const int w = it & ((1 << per_entry_log) - 1);
    const int blk = w >> s, j = w & (S - 1);
    uint32_t* base = lds + e * lds_stride;
    const int pos0 = (blk << (s + r)) + j;
    uint32_t x[R];
#pragma unroll
    for (int u = 0; u < R; ++u) x[u] = base[lds_pos(pos0 + u * S)];
    const Tw* t = tw + j * (R - 1);
#pragma unroll
    for (int v = r - 1; v >= 0; --v) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        if (u & (1 << v)) continue;
        const int u2 = u | (1 << v);
        const Tw tt = t[(1 << v) - 1 + (u & ((1 << v) - 1))];
        const uint32_t a0 = x[u], b0 = x[u2];
        x[u] = add_mod(a0, b0, q);
        x[u2] = mul_shoup(a0 + (q - b0), tt.w, tt.wp, q);
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) base[lds_pos(pos0 + u * S)] = x[u];
  }
}

// One decimation-in-time pass of r stages at stride 2^s.
template <int r>
__device__ __forceinline__ void dit_pass(uint32_t* lds, int lds_stride, int logL, int s,
                                         const Tw* __restrict__ tw, int eb_log, uint32_t q) {
  constexpr int R = 1 << r;
  const int S = 1 << s;
  const int per_entry_log = logL - r;
  const int items = 1 << (per_entry_log + eb_log);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int e = it >> per_entry_log;
    const int w = it & ((1 << per_entry_log) - 1);
    const int blk = w >> s, j = w & (S - 1);
    uint32_t* base = lds + e * lds_stride;
    const int pos0 = (blk << (s + r)) + j;
    uint32_t x[R];
#pragma unroll
    for (int u = 0; u < R; ++u) x[u] = base[lds_pos(pos0 + u * S)];
    const Tw* t = tw + j * (R - 1);
#pragma unroll
    for (int v = 0; v < r; ++v) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        if (u & (1 << v)) continue;
        const int u2 = u | (1 << v);
        const Tw tt = t[(1 << v) - 1 + (u & ((1 << v) - 1))];
        const uint32_t a0 = x[u];
        const uint32_t b0 = mul_shoup(x[u2], tt.w, tt.wp, q);
        x[u] = add_mod(a0, b0, q);
        x[u2] = sub_mod(a0, b0, q);
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) base[lds_pos(pos0 + u * S)] = x[u];
  }
}

__device__ __forceinline__ void run_dif(const NttLaunch& a, uint32_t* lds, const PrimeConst& P) {
  for (int ps = 0; ps < a.npass; ++ps) {
    const Tw* tw = P.tw_fwd + a.tw_off[ps];
    switch (a.stages[ps]) {
      case 1: dif_pass<1>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
      case 2: dif_pass<2>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
      case 3: dif_pass<3>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
      case 4: dif_pass<4>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
      default: dif_pass<5>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void run_dit(const NttLaunch& a, uint32_t* lds, const PrimeConst& P) {
  for (int ps = a.npass - 1; ps >= 0; --ps) {
    const Tw* tw = P.tw_inv + a.tw_off[ps];
    switch (a.stages[ps]) {
      case 1: dit_pass<1>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
      case 2: dit_pass<2>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
      case 3: dit_pass<3>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
      case 4: dit_pass<4>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
      default: dit_pass<5>(lds, a.lds_stride, a.logL, a.stride_log[ps], tw, a.eb_log, P.q); break;
    }
    __syncthreads();
  }
}

template <typename TIn, bool REDUCE>
__global__ __launch_bounds__(256) void ntt_fwd_kernel(NttLaunch a) {
  extern __shared__ uint32_t lds[];
  const int prime = blockIdx.y;
  const PrimeConst& P = a.pc[prime];
  const uint32_t q = P.q;
  const int L = 1 << a.logL;
  const int EB = 1 << a.eb_log;
  const int e0 = blockIdx.x * EB;
  const TIn* in = (const TIn*)a.in + a.in_prime_stride * prime;
  const int total = L << a.eb_log;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int c = idx >> a.eb_log, e = idx & (EB - 1);
    uint32_t v = 0;
    if (c < a.nin && e0 + e < a.E) {
      const TIn x = in[(size_t)c * a.E + e0 + e];
      v = REDUCE ? reduce_u64((uint64_t)x, q, P.mu) : (uint32_t)x;
    }
    lds[e * a.lds_stride + lds_pos(c)] = v;
  }
  __syncthreads();
  run_dif(a, lds, P);
  uint32_t* out = (uint32_t*)a.out + a.out_prime_stride * prime;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int t = idx >> a.eb_log, e = idx & (EB - 1);
    if (e0 + e < a.E) out[(size_t)t * a.E + e0 + e] = lds[e * a.lds_stride + lds_pos(t)];
  }
}

template <typename TOut>
__global__ __launch_bounds__(256) void ntt_inv_kernel(NttLaunch a) {
  extern __shared__ uint32_t lds[];
  const int prime = blockIdx.y;
  const PrimeConst& P = a.pc[prime];
  const int L = 1 << a.logL;
  const int EB = 1 << a.eb_log;
  const int e0 = blockIdx.x * EB;
  const uint32_t* in = (const uint32_t*)a.in + a.in_prime_stride * prime;
  const int total = L << a.eb_log;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int t = idx >> a.eb_log, e = idx & (EB - 1);
    uint32_t v = 0;
    if (e0 + e < a.E) v = in[(size_t)t * a.E + e0 + e];
    lds[e * a.lds_stride + lds_pos(t)] = v;
  }
  __syncthreads();
  run_dit(a, lds, P);
  TOut* out = (TOut*)a.out + a.out_prime_stride * prime;
  const int nout = a.nin << a.eb_log;
  for (int idx = threadIdx.x; idx < nout; idx += blockDim.x) {
    const int c = idx >> a.eb_log, e = idx & (EB - 1);
    if (e0 + e < a.E) out[(size_t)c * a.E + e0 + e] = (TOut)lds[e * a.lds_stride + lds_pos(c)];
  }
}

// ---- host side ---------------------------------------------------------------

static int entries_log_per_block(int logL) {
  // about 16K residues (64 KiB) of LDS per workgroup, at least one entry
  int eb = 14 - logL;
  return eb < 0 ? 0 : eb;
}

void fill_ntt_launch(NttLaunch* a, int logL, int E, int nin) {
  const PassPlan PP = make_pass_plan(logL);
  a->logL = logL;
  a->npass = PP.npass;
  for (int i = 0; i < kMaxPasses; ++i) {
    a->stages[i] = i < PP.npass ? PP.stages[i] : 0;
    a->stride_log[i] = i < PP.npass ? PP.stride_log[i] : 0;
    a->tw_off[i] = i < PP.npass ? PP.tw_off[i] : 0;
  }
  a->nin = nin;
  a->E = E;
  int eb = entries_log_per_block(logL);
  while (eb > 0 && (1 << (eb - 1)) >= E) --eb;  // no more slots than entries
  a->eb_log = eb;
  const int L = 1 << logL;
  a->lds_stride = L + (L >> 5) + 1;
}

static size_t lds_bytes(const NttLaunch& a) {
  return sizeof(uint32_t) * (size_t)a.lds_stride << a.eb_log;
}

template <typename K>
static int launch(K kernel, const NttLaunch& a, int nprimes, hipStream_t s) {
  const size_t lds = lds_bytes(a);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int EB = 1 << a.eb_log;
  dim3 grid((a.E + EB - 1) / EB, nprimes);
  hipLaunchKernelGGL(kernel, grid, dim3(256), lds, s, a);
  return hipGetLastError();
}

int launch_ntt_fwd(const NttLaunch& a, int elem_bytes, int reduce, int nprimes,
                   hipStream_t s) {
  if (elem_bytes == 8) return launch(ntt_fwd_kernel<uint64_t, true>, a, nprimes, s);
  if (reduce) return launch(ntt_fwd_kernel<uint32_t, true>, a, nprimes, s);
  return launch(ntt_fwd_kernel<uint32_t, false>, a, nprimes, s);
}

int launch_ntt_inv(const NttLaunch& a, int out_elem_bytes, int nprimes, hipStream_t s) {
  if (out_elem_bytes == 8) return launch(ntt_inv_kernel<uint64_t>, a, nprimes, s);
  return launch(ntt_inv_kernel<uint32_t>, a, nprimes, s);
}

}  // namespace pm
