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
// Shoup's precomputed quotient (pm_arith.h); the 2^r - 1 twiddles a thread
// needs in a pass are stored slot-major, so the lanes of a wave (consecutive
// j) read consecutive pairs.  Residues stay canonical ([0, q)) between stages,
// because 2q < 2^32 but 4q may not be (q can exceed 2^30).
//
// Forward = decimation in frequency on natural-order input: position t of the
// output holds the value at w^bitrev(t).  Inverse = decimation in time on that
// order with w^-1, giving L times the natural-order coefficients.
#include <stdlib.h>

#include "pm_arith.h"
#include "pm_kernels.h"

namespace pm {

__device__ __forceinline__ int lds_pos(int pos) { return pos + (pos >> 5); }

// Items of a pass: a thread takes one (blk, j) position group and EPI entries;
// it loads the 2^r - 1 twiddles of its j once, up front, and applies them to
// all EPI entries (twiddles do not depend on the entry).
template <int r, int EPI, bool DIF>
__device__ __forceinline__ void ntt_pass(uint32_t* lds, int lds_stride, int logL, int s,
                                         const Tw* __restrict__ tw, int eb_log, uint32_t q) {
  constexpr int R = 1 << r;
  constexpr int epi_log = EPI == 4 ? 2 : EPI == 2 ? 1 : 0;
  const int S = 1 << s;
  const int per_entry_log = logL - r;
  const int items = 1 << (per_entry_log + eb_log - epi_log);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int eg = it >> per_entry_log;
    const int w = it & ((1 << per_entry_log) - 1);
    const int blk = w >> s, j = w & (S - 1);
    const int pos0 = (blk << (s + r)) + j;
    Tw t[R - 1];
#pragma unroll
    for (int k = 0; k < R - 1; ++k) t[k] = tw[k * S + j];
#pragma unroll
    for (int ee = 0; ee < EPI; ++ee) {
      uint32_t* base = lds + ((eg << epi_log) + ee) * lds_stride;
      uint32_t x[R];
#pragma unroll
      for (int u = 0; u < R; ++u) x[u] = base[lds_pos(pos0 + u * S)];
      if (DIF) {
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
      } else {
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
      }
#pragma unroll
      for (int u = 0; u < R; ++u) base[lds_pos(pos0 + u * S)] = x[u];
    }
  }
}

// Entries per item: enough that the block's 256 threads have about one item
// each, at most the entries the block holds, at most 2.
__device__ __forceinline__ int pass_epi(int logL, int r, int eb_log) {
  const int triples_log = logL - r + eb_log;
  int epi_log = triples_log - 8;
  if (epi_log > eb_log) epi_log = eb_log;
  if (epi_log > 1) epi_log = 1;
  return epi_log < 0 ? 0 : epi_log;
}

template <bool DIF, int r>
__device__ __forceinline__ void pass_r(const NttLaunch& a, uint32_t* lds, const Tw* tw,
                                       int s, uint32_t q) {
  if (pass_epi(a.logL, r, a.eb_log) == 1)
    ntt_pass<r, 2, DIF>(lds, a.lds_stride, a.logL, s, tw, a.eb_log, q);
  else
    ntt_pass<r, 1, DIF>(lds, a.lds_stride, a.logL, s, tw, a.eb_log, q);
}

template <bool DIF>
__device__ __forceinline__ void run_pass(const NttLaunch& a, uint32_t* lds, const Tw* tw,
                                         int ps, uint32_t q) {
  const int s = a.stride_log[ps];
  switch (a.stages[ps]) {
    case 1: pass_r<DIF, 1>(a, lds, tw, s, q); break;
    case 2: pass_r<DIF, 2>(a, lds, tw, s, q); break;
    case 3: pass_r<DIF, 3>(a, lds, tw, s, q); break;
    case 4: pass_r<DIF, 4>(a, lds, tw, s, q); break;
    default: pass_r<DIF, 5>(a, lds, tw, s, q); break;
  }
}

__device__ __forceinline__ void run_dif(const NttLaunch& a, uint32_t* lds, const PrimeConst& P) {
  for (int ps = 0; ps < a.npass; ++ps) {
    run_pass<true>(a, lds, P.tw_fwd + a.tw_off[ps], ps, P.q);
    __syncthreads();
  }
}

__device__ __forceinline__ void run_dit(const NttLaunch& a, uint32_t* lds, const PrimeConst& P) {
  for (int ps = a.npass - 1; ps >= 0; --ps) {
    run_pass<false>(a, lds, P.tw_inv + a.tw_off[ps], ps, P.q);
    __syncthreads();
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumber them so that consecutive entry blocks, which share cache
// lines of the coefficient-major input and point-major output, run on the
// same XCD.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int nx = 8;
  const int q = nb / nx, r = nb % nx;
  const int x = b % nx, i = b / nx;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <typename T, int V>
struct alignas(sizeof(T) * V) Vec {
  T v[V];
};

template <typename TIn, bool REDUCE, int V>
__global__ __launch_bounds__(256, 2) void ntt_fwd_kernel(NttLaunch a) {
  extern __shared__ uint32_t lds[];
  const int prime = blockIdx.y;
  const PrimeConst& P = a.pc[prime];
  const uint32_t q = P.q;
  const int EB = 1 << a.eb_log;
  const int e0 = xcd_block(blockIdx.x, gridDim.x) * EB;
  const TIn* in = (const TIn*)a.in + a.in_prime_stride * prime;
  const int glog = a.eb_log - (V == 4 ? 2 : V == 2 ? 1 : 0);  // vector groups per row
  const int total = 1 << (a.logL + glog);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int c = idx >> glog, e = (idx & ((1 << glog) - 1)) * V;
    Vec<TIn, V> x;
    if (c < a.nin && e0 + e < a.E) {
      x = *(const Vec<TIn, V>*)(in + (size_t)c * a.E + e0 + e);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) x.v[v] = 0;
    }
#pragma unroll
    for (int v = 0; v < V; ++v)
      lds[(e + v) * a.lds_stride + lds_pos(c)] =
          REDUCE ? reduce_u64((uint64_t)x.v[v], q, P.mu) : (uint32_t)x.v[v];
  }
  __syncthreads();
  run_dif(a, lds, P);
  uint32_t* out = (uint32_t*)a.out + a.out_prime_stride * prime;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int t = idx >> glog, e = (idx & ((1 << glog) - 1)) * V;
    if (e0 + e < a.E) {
      Vec<uint32_t, V> y;
#pragma unroll
      for (int v = 0; v < V; ++v) y.v[v] = lds[(e + v) * a.lds_stride + lds_pos(t)];
      *(Vec<uint32_t, V>*)(out + (size_t)t * a.E + e0 + e) = y;
    }
  }
}

template <typename TOut, int V>
__global__ __launch_bounds__(256, 2) void ntt_inv_kernel(NttLaunch a) {
  extern __shared__ uint32_t lds[];
  const int prime = blockIdx.y;
  const PrimeConst& P = a.pc[prime];
  const int EB = 1 << a.eb_log;
  const int e0 = xcd_block(blockIdx.x, gridDim.x) * EB;
  const uint32_t* in = (const uint32_t*)a.in + a.in_prime_stride * prime;
  const int glog = a.eb_log - (V == 4 ? 2 : V == 2 ? 1 : 0);
  const int total = 1 << (a.logL + glog);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int t = idx >> glog, e = (idx & ((1 << glog) - 1)) * V;
    Vec<uint32_t, V> x;
    if (e0 + e < a.E) {
      x = *(const Vec<uint32_t, V>*)(in + (size_t)t * a.E + e0 + e);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) x.v[v] = 0;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) lds[(e + v) * a.lds_stride + lds_pos(t)] = x.v[v];
  }
  __syncthreads();
  run_dit(a, lds, P);
  TOut* out = (TOut*)a.out + a.out_prime_stride * prime;
  const int nout = a.nin << glog;
  for (int idx = threadIdx.x; idx < nout; idx += blockDim.x) {
    const int c = idx >> glog, e = (idx & ((1 << glog) - 1)) * V;
    if (e0 + e < a.E) {
      Vec<TOut, V> y;
#pragma unroll
      for (int v = 0; v < V; ++v) y.v[v] = (TOut)lds[(e + v) * a.lds_stride + lds_pos(c)];
      *(Vec<TOut, V>*)(out + (size_t)c * a.E + e0 + e) = y;
    }
  }
}

// ---- host side ---------------------------------------------------------------

static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v && *v ? atoi(v) : dflt;
}

// log2 of the entries one workgroup transforms.  Tuning knob
// PM_TUNE_NTT_LDS_LOG: log2 of the residues held in LDS per workgroup
// (default 14, i.e. 64 KiB, two workgroups per CU).
static int entries_log_per_block(int logL) {
  static const int lds_log = env_int("PM_TUNE_NTT_LDS_LOG", 14);
  int eb = lds_log - logL;
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
  // Entries move between HBM and LDS in vectors of V consecutive residues.
  int v = 4;
  while (v > 1 && ((E % v) != 0 || (1 << eb) % v != 0)) v >>= 1;
  a->vec = v;
  const int L = 1 << logL;
  a->lds_stride = L + (L >> 5) + 1;
}

static size_t lds_bytes(const NttLaunch& a) {
  return sizeof(uint32_t) * (size_t)a.lds_stride << a.eb_log;
}

template <typename K>
static int launch(K kernel, const NttLaunch& a, int nprimes, hipStream_t s) {
  const size_t lds = lds_bytes(a);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
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

template <typename TIn, bool REDUCE>
static int launch_fwd_v(const NttLaunch& a, int nprimes, hipStream_t s) {
  // 64-bit inputs move in vectors of at most 16 bytes
  if (a.vec == 4 && sizeof(TIn) == 4) return launch(ntt_fwd_kernel<TIn, REDUCE, 4>, a, nprimes, s);
  if (a.vec == 4) return launch(ntt_fwd_kernel<TIn, REDUCE, 2>, a, nprimes, s);
  if (a.vec == 2) return launch(ntt_fwd_kernel<TIn, REDUCE, 2>, a, nprimes, s);
  return launch(ntt_fwd_kernel<TIn, REDUCE, 1>, a, nprimes, s);
}

int launch_ntt_fwd(const NttLaunch& a, int elem_bytes, int reduce, int nprimes,
                   hipStream_t s) {
  if (elem_bytes == 8) return launch_fwd_v<uint64_t, true>(a, nprimes, s);
  if (reduce) return launch_fwd_v<uint32_t, true>(a, nprimes, s);
  return launch_fwd_v<uint32_t, false>(a, nprimes, s);
}

template <typename TOut>
static int launch_inv_v(const NttLaunch& a, int nprimes, hipStream_t s) {
  if (a.vec == 4 && sizeof(TOut) == 4) return launch(ntt_inv_kernel<TOut, 4>, a, nprimes, s);
  if (a.vec == 4) return launch(ntt_inv_kernel<TOut, 2>, a, nprimes, s);
  if (a.vec == 2) return launch(ntt_inv_kernel<TOut, 2>, a, nprimes, s);
  return launch(ntt_inv_kernel<TOut, 1>, a, nprimes, s);
}

int launch_ntt_inv(const NttLaunch& a, int out_elem_bytes, int nprimes, hipStream_t s) {
  if (out_elem_bytes == 8) return launch_inv_v<uint64_t>(a, nprimes, s);
  return launch_inv_v<uint32_t>(a, nprimes, s);
}

}  // namespace pm
