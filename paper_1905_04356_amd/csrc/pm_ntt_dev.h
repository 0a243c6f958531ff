// pm_ntt_dev.h -- device side of the batched number-theoretic transforms.
//
// Evaluation at the L-th roots of unity of an FFT prime q and interpolation
// back (Hyun, Neiger, Schost, ISSAC 2019, Section 2, "Polynomial
// multiplication" (FFT paragraph) and "Polynomial matrix multiplication"
// (evaluation/interpolation at roots of unity for FFT primes)).
//
// Forward = decimation in frequency on natural-order input: position t of the
// output holds the value at w^bitrev(t).  Inverse = decimation in time on that
// order with w^-1, giving L times the natural-order coefficients (the
// pointwise kernel applies L^{-1}).  Residues stay canonical ([0, q)) between
// stages, because 2q < 2^32 but 4q may not be (q can exceed 2^30).
// Multiplication by a root of unity uses Shoup's precomputed quotient
// (pm_arith.h).
//
// Data layout in HBM: inputs are coefficient-major X[c][e] and evaluations
// point-major Xhat[t][e] (e = entry), so a transform reads and writes rows of
// consecutive entries.  Two kernel shapes:
//   * LDS kernel: a workgroup holds 2^eb_log entries x 2^blk_log positions in
//     LDS and runs passes of up to 4 radix-2 stages; in a pass a thread
//     loads 2^r values at stride S into registers, runs r stages there and
//     writes them back.  The 2^r - 1 twiddles a thread needs are stored
//     slot-major (consecutive j read consecutive pairs), loaded once per
//     item and applied to every entry of the item.
//   * Column kernel (split > 0): the first forward pass (last inverse pass),
//     of stride S = L / 2^split, streams rows straight from HBM to HBM with
//     one thread per (j, entry), so every row access is a contiguous run of
//     entries.  The remaining passes act on independent blocks of S
//     consecutive positions; the LDS kernel then holds many entries of one
//     block and transforms it in place.
#pragma once
#include <utility>

#include "pm_arith.h"
#include "pm_crt_dev.h"
#include "pm_kernels.h"

namespace pm {

constexpr int kNT = 512;      // threads of the LDS kernels
constexpr int kColNT = 256;   // threads of the single-product column kernel

__device__ __forceinline__ int lds_pos(int pos) { return pos + (pos >> 5); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Renumber them so that consecutive entry blocks, which share cache
// lines of the row-major buffers, run on the same XCD.
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

// A load marked non-temporal (read once: it should not displace data that
// is read again from the last-level cache).
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> load_nt(const Vec<T, V>* p) {
  constexpr int W = sizeof(T) * V / 4;
  static_assert(W == 1 || W == 2 || W == 4 || W == 8, "load_nt: 4- to 32-byte vectors");
  typedef uint32_t W4 __attribute__((ext_vector_type(4)));
  typedef uint32_t W2 __attribute__((ext_vector_type(2)));
  Vec<T, V> r;
  if constexpr (W == 8) {  // two 16-byte halves
    const W4 x0 = __builtin_nontemporal_load((const W4*)p);
    const W4 x1 = __builtin_nontemporal_load((const W4*)p + 1);
    __builtin_memcpy(&r, &x0, sizeof x0);
    __builtin_memcpy((char*)&r + sizeof x0, &x1, sizeof x1);
  } else if constexpr (W == 4) {
    const W4 x = __builtin_nontemporal_load((const W4*)p);
    __builtin_memcpy(&r, &x, sizeof r);
  } else if constexpr (W == 2) {
    const W2 x = __builtin_nontemporal_load((const W2*)p);
    __builtin_memcpy(&r, &x, sizeof r);
  } else {
    const uint32_t x = __builtin_nontemporal_load((const uint32_t*)p);
    __builtin_memcpy(&r, &x, sizeof r);
  }
  return r;
}

// r radix-2 stages on x[0..2^r) held in registers.  DIF: stage distance
// 2^v for v = r-1 .. 0, (a, b) -> (a + b, (a - b) w).  DIT: v = 0 .. r-1,
// (a, b) -> (a + b w, a - b w).  ZHI (DIF only): x[2^(r-1) ..] are zero, so
// the first stage is (a, 0) -> (a, a w).  t[(2^v - 1) + u'] is the twiddle of
// stage v for butterflies whose lower index is u' mod 2^v.  UNIT0: the
// butterflies run at stride 1 of the whole transform, where the twiddle of
// lower index 0 is w^0 = 1 in every stage, so those take no product (half
// of the last stage, a quarter of the one before, ...).
// LAZY (moduli with 4q < 2^32): Harvey's lazy butterflies (D. Harvey,
// "Faster arithmetic for number-theoretic transforms", 2014): values stay in
// [0, 2q) instead of [0, q).  A sum a + b < 4q is brought back below 2q, a
// difference enters the product as a + 2q - b < 4q, and the products skip
// their final correction (Shoup's product of any 32-bit value is below 2q):
// 8 instead of 10 operations per forward butterfly, 10 instead of 11 per
// inverse one.
template <int r, bool DIF, bool ZHI, bool UNIT0 = false, bool LAZY = false>
__device__ __forceinline__ void butterflies(uint32_t* x, const Tw* t, uint32_t q) {
  constexpr int R = 1 << r;
  const uint32_t nq = opaque_neg(q);
  if (LAZY) {
    const uint32_t q2 = 2 * q;
    if (DIF) {
#pragma unroll
      for (int v = r - 1; v >= 0; --v) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
          if (u & (1 << v)) continue;
          const int u2 = u | (1 << v);
          const int ul = u & ((1 << v) - 1);
          const uint32_t a0 = x[u], b0 = x[u2];
          x[u] = reduce_once(a0 + b0, q2);
          if (UNIT0 && ul == 0) {
            x[u2] = reduce_once(a0 + (q2 - b0), q2);
          } else {
            const Tw tt = t[(1 << v) - 1 + ul];
            x[u2] = mul_shoup_lazy_nq(a0 + (q2 - b0), tt.w, tt.wp, nq);
          }
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < r; ++v) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
          if (u & (1 << v)) continue;
          const int u2 = u | (1 << v);
          const int ul = u & ((1 << v) - 1);
          const uint32_t a0 = x[u];
          uint32_t b0 = x[u2];
          if (!(UNIT0 && ul == 0)) {
            const Tw tt = t[(1 << v) - 1 + ul];
            b0 = mul_shoup_lazy_nq(b0, tt.w, tt.wp, nq);
          }
          x[u] = reduce_once(a0 + b0, q2);
          x[u2] = reduce_once(a0 + (q2 - b0), q2);
        }
      }
    }
    return;
  }
  if (DIF) {
#pragma unroll
    for (int v = r - 1; v >= 0; --v) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        if (u & (1 << v)) continue;
        const int u2 = u | (1 << v);
        const int ul = u & ((1 << v) - 1);
        if (UNIT0 && ul == 0) {
          const uint32_t a0 = x[u], b0 = x[u2];
          x[u] = add_mod(a0, b0, q);
          x[u2] = sub_mod(a0, b0, q);
          continue;
        }
        const Tw tt = t[(1 << v) - 1 + ul];
        if (ZHI && v == r - 1) {
          x[u2] = mul_shoup_nq(x[u], tt.w, tt.wp, q, nq);
        } else {
          const uint32_t a0 = x[u], b0 = x[u2];
          x[u] = add_mod(a0, b0, q);
          x[u2] = mul_shoup_nq(a0 + (q - b0), tt.w, tt.wp, q, nq);
        }
      }
    }
  } else {
#pragma unroll
    for (int v = 0; v < r; ++v) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        if (u & (1 << v)) continue;
        const int u2 = u | (1 << v);
        const int ul = u & ((1 << v) - 1);
        const uint32_t a0 = x[u];
        uint32_t b0 = x[u2];
        if (!(UNIT0 && ul == 0)) {
          const Tw tt = t[(1 << v) - 1 + ul];
          b0 = mul_shoup_nq(b0, tt.w, tt.wp, q, nq);
        }
        x[u] = add_mod(a0, b0, q);
        x[u2] = sub_mod(a0, b0, q);
      }
    }
  }
}

// One pass of r stages at stride 2^s over LDS blocks of 2^glog positions.
// Items: a thread takes one (blk, j) position group and EPI entries; it loads
// the 2^r - 1 twiddles of its j once and applies them to all EPI entries.
template <int r, int EPI, bool DIF, bool ZHI>
__device__ __forceinline__ void lds_pass(uint32_t* lds, int lds_stride, int glog, int s,
                                         const Tw* __restrict__ tw, int eb_log, uint32_t q) {
  constexpr int R = 1 << r;
  constexpr int epi_log = EPI == 2 ? 1 : 0;
  const int S = 1 << s;
  const int per_entry_log = glog - r;
  const int items = 1 << (per_entry_log + eb_log - epi_log);
  for (int it = threadIdx.x; it < items; it += kNT) {
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
      for (int u = 0; u < R; ++u)
        x[u] = (ZHI && u >= R / 2) ? 0u : base[lds_pos(pos0 + u * S)];
      butterflies<r, DIF, ZHI>(x, t, q);
#pragma unroll
      for (int u = 0; u < R; ++u) base[lds_pos(pos0 + u * S)] = x[u];
    }
  }
}

// Entries per item: enough that the block's threads have about one item
// each, at most the entries the block holds, at most 2.
__device__ __forceinline__ int pass_epi(int glog, int r, int eb_log) {
  int epi_log = glog - r + eb_log - 9;  // 2^9 = kNT
  if (epi_log > eb_log) epi_log = eb_log;
  if (epi_log > 1) epi_log = 1;
  return epi_log < 0 ? 0 : epi_log;
}

template <bool DIF, bool ZHI, int r>
__device__ __forceinline__ void pass_r(const NttLaunch& a, uint32_t* lds, const Tw* tw, int glog,
                                       int s, uint32_t q) {
  if (pass_epi(glog, r, a.eb_log) == 1)
    lds_pass<r, 2, DIF, ZHI>(lds, a.lds_stride, glog, s, tw, a.eb_log, q);
  else
    lds_pass<r, 1, DIF, ZHI>(lds, a.lds_stride, glog, s, tw, a.eb_log, q);
}

template <bool DIF, bool ZHI>
__device__ __forceinline__ void run_pass(const NttLaunch& a, uint32_t* lds, const Tw* tw,
                                         int glog, int ps, uint32_t q) {
  const int s = a.stride_log[ps];
  switch (a.stages[ps]) {
    case 1: pass_r<DIF, ZHI, 1>(a, lds, tw, glog, s, q); break;
    case 2: pass_r<DIF, ZHI, 2>(a, lds, tw, glog, s, q); break;
    case 3: pass_r<DIF, ZHI, 3>(a, lds, tw, glog, s, q); break;
    default: pass_r<DIF, ZHI, 4>(a, lds, tw, glog, s, q); break;
  }
}

// ---- tiles ------------------------------------------------------------------
// Each function below is the work of one workgroup; the single-product
// kernels and the batched phase kernels both call them.  eb = entry block
// index, z = position block index (split transforms).

// Unsplit forward transform: coefficient-major input (rows < nin, nin <= L/2
// unless L == 1) to point-major output.
template <typename TIn, bool REDUCE, int V>
__device__ __forceinline__ void fwd_lds_tile(const NttLaunch& a, int prime, int eb,
                                             uint32_t* lds) {
  const PrimeConst& P = a.pc[prime];
  const uint32_t q = P.q;
  const int EB = 1 << a.eb_log;
  const int e0 = eb * EB;
  const TIn* in = (const TIn*)a.in + a.in_prime_stride * prime;
  const int glog = a.eb_log - (V == 4 ? 2 : V == 2 ? 1 : 0);  // vector groups per row
  const int total = 1 << (a.logL + glog);
  // rows at or beyond L/2 are never read by the first pass when nin <= L/2
  const bool zhi = a.npass > 0 && 2 * a.nin <= (1 << a.logL);
  const int ltotal = 1 << ((zhi ? a.logL - 1 : a.logL) + glog);
  for (int idx = threadIdx.x; idx < ltotal; idx += kNT) {
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
  for (int ps = 0; ps < a.npass; ++ps) {
    if (ps == 0 && zhi)
      run_pass<true, true>(a, lds, P.tw_fwd + a.tw_off[ps], a.logL, ps, q);
    else
      run_pass<true, false>(a, lds, P.tw_fwd + a.tw_off[ps], a.logL, ps, q);
    __syncthreads();
  }
  uint32_t* out = (uint32_t*)a.out + a.out_prime_stride * prime;
  for (int idx = threadIdx.x; idx < total; idx += kNT) {
    const int t = idx >> glog, e = (idx & ((1 << glog) - 1)) * V;
    if (e0 + e < a.E) {
      Vec<uint32_t, V> y;
#pragma unroll
      for (int v = 0; v < V; ++v) y.v[v] = lds[(e + v) * a.lds_stride + lds_pos(t)];
      *(Vec<uint32_t, V>*)(out + (size_t)t * a.E + e0 + e) = y;
    }
  }
}

// Unsplit inverse transform: point-major input to coefficient-major output
// (coefficients out_lo .. out_lo + nin - 1 to rows 0 .. nin - 1).
template <typename TOut, int V>
__device__ __forceinline__ void inv_lds_tile(const NttLaunch& a, int prime, int eb,
                                             uint32_t* lds) {
  const PrimeConst& P = a.pc[prime];
  const int EB = 1 << a.eb_log;
  const int e0 = eb * EB;
  const uint32_t* in = (const uint32_t*)a.in + a.in_prime_stride * prime;
  const int glog = a.eb_log - (V == 4 ? 2 : V == 2 ? 1 : 0);
  const int total = 1 << (a.logL + glog);
  for (int idx = threadIdx.x; idx < total; idx += kNT) {
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
  for (int ps = a.npass - 1; ps >= 0; --ps) {
    run_pass<false, false>(a, lds, P.tw_inv + a.tw_off[ps], a.logL, ps, P.q);
    __syncthreads();
  }
  TOut* out = (TOut*)a.out + a.out_prime_stride * prime;
  const int nout = a.nin << glog;
  for (int idx = threadIdx.x; idx < nout; idx += kNT) {
    const int c = idx >> glog, e = (idx & ((1 << glog) - 1)) * V;
    if (e0 + e < a.E) {
      Vec<TOut, V> y;
#pragma unroll
      for (int v = 0; v < V; ++v)
        y.v[v] = (TOut)lds[(e + v) * a.lds_stride + lds_pos(c + a.out_lo)];
      *(Vec<TOut, V>*)(out + (size_t)c * a.E + e0 + e) = y;
    }
  }
}

// Split transforms, LDS part: block z of 2^blk_log consecutive positions of
// the point-major buffer `out`, transformed in place by passes 1 .. npass-1
// (forward, DIF) or npass-1 .. 1 (inverse, DIT).
//
// The tile sits in LDS position-major, as in HBM: position t, entry e at word
// t * pitch + e.  Rows move between HBM and LDS as whole vectors, and a pass
// item takes EPI adjacent entries at its 2^r positions pos0 + u S, one vector
// access per position.  Consecutive lanes take consecutive entry groups of
// the same position group, so they share the twiddles of that group and
// their LDS addresses differ by a constant.
template <int r, int EPI, bool DIF, int NT>
__device__ __forceinline__ void block_pass(uint32_t* lds, int pitch, int blk_log, int eb_log,
                                           int s, const Tw* __restrict__ tw, uint32_t q) {
  constexpr int R = 1 << r;
  constexpr int epi_log = EPI == 4 ? 2 : EPI == 2 ? 1 : 0;
  const int S = 1 << s;
  const int glog = eb_log - epi_log;  // log2 entry groups per position
  const int items = 1 << (blk_log - r + glog);
  const int ustep = S * pitch;
  for (int it = threadIdx.x; it < items; it += NT) {
    const int g = it & ((1 << glog) - 1);
    const int w = it >> glog;
    const int blk = w >> s, j = w & (S - 1);
    uint32_t* base = lds + ((blk << (s + r)) + j) * pitch + g * EPI;
    Tw t[R - 1];
#pragma unroll
    for (int k = 0; k < R - 1; ++k) t[k] = tw[k * S + j];
    uint32_t x[EPI][R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const Vec<uint32_t, EPI> v = *(const Vec<uint32_t, EPI>*)(base + u * ustep);
#pragma unroll
      for (int c = 0; c < EPI; ++c) x[c][u] = v.v[c];
    }
#pragma unroll
    for (int c = 0; c < EPI; ++c) butterflies<r, DIF, false>(x[c], t, q);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      Vec<uint32_t, EPI> v;
#pragma unroll
      for (int c = 0; c < EPI; ++c) v.v[c] = x[c][u];
      *(Vec<uint32_t, EPI>*)(base + u * ustep) = v;
    }
  }
}

// Entries per pass item: the widest vector (<= 4, <= the entries of the
// tile) that still gives every one of the 2^nt_log threads an item.
__device__ __forceinline__ int block_epi_log(int blk_log, int eb_log, int r, int nt_log) {
  int e = eb_log < 2 ? eb_log : 2;
  while (e > 0 && blk_log - r + eb_log - e < nt_log) --e;
  return e;
}

template <int r, bool DIF, int NT, int MAXEPI>
__device__ __forceinline__ void block_pass_r(const NttLaunch& a, uint32_t* lds, const Tw* tw,
                                             int ps, uint32_t q) {
  const int s = a.stride_log[ps];
  // (16 residues x 4 entries would not fit the register budget of 4 waves
  // per SIMD; with MAXEPI < 4 radix-16 items take a single entry)
  constexpr int EPI2 = (r == 4 && MAXEPI < 4) ? 1 : 2;
  switch (block_epi_log(a.blk_log, a.eb_log, r, NT == 256 ? 8 : 9)) {
    case 2:
      block_pass<r, (r < 4 && MAXEPI >= 4) ? 4 : EPI2, DIF, NT>(lds, a.blk_pitch, a.blk_log,
                                                                a.eb_log, s, tw, q);
      break;
    case 1: block_pass<r, EPI2, DIF, NT>(lds, a.blk_pitch, a.blk_log, a.eb_log, s, tw, q); break;
    default: block_pass<r, 1, DIF, NT>(lds, a.blk_pitch, a.blk_log, a.eb_log, s, tw, q); break;
  }
}

template <bool DIF, int NT, int MAXEPI>
__device__ __forceinline__ void block_run_pass(const NttLaunch& a, uint32_t* lds, const Tw* tw,
                                               int ps, uint32_t q) {
  switch (a.stages[ps]) {
    case 1: block_pass_r<1, DIF, NT, MAXEPI>(a, lds, tw, ps, q); break;
    case 2: block_pass_r<2, DIF, NT, MAXEPI>(a, lds, tw, ps, q); break;
    case 3: block_pass_r<3, DIF, NT, MAXEPI>(a, lds, tw, ps, q); break;
    default: block_pass_r<4, DIF, NT, MAXEPI>(a, lds, tw, ps, q); break;
  }
}

// One tile with NT threads (512 in the batched phase kernels; the
// single-product kernel may use 256 so that more tiles share a CU) and at
// most MAXEPI entries per pass item (the batched kernels use 2, and 1 for
// radix-16 passes, to stay within their register budget).
template <bool DIF, int V, int NT = kNT, int MAXEPI = 4>
__device__ __forceinline__ void block_tile(const NttLaunch& a, int prime, int eb, int z,
                                           uint32_t* lds) {
  const PrimeConst& P = a.pc[prime];
  const int EB = 1 << a.eb_log;
  const int e0 = eb * EB;
  const int pitch = a.blk_pitch;
  uint32_t* buf = (uint32_t*)a.out + a.out_prime_stride * prime + ((size_t)z << a.blk_log) * a.E;
  const int glog = a.eb_log - (V == 4 ? 2 : V == 2 ? 1 : 0);
  const int total = 1 << (a.blk_log + glog);
  for (int idx = threadIdx.x; idx < total; idx += NT) {
    const int t = idx >> glog, e = (idx & ((1 << glog) - 1)) * V;
    Vec<uint32_t, V> x;
    if (e0 + e < a.E) {
      x = *(const Vec<uint32_t, V>*)(buf + (size_t)t * a.E + e0 + e);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) x.v[v] = 0;
    }
    *(Vec<uint32_t, V>*)(lds + t * pitch + e) = x;
  }
  __syncthreads();
  if (DIF) {
    for (int ps = 1; ps < a.npass; ++ps) {
      block_run_pass<true, NT, MAXEPI>(a, lds, P.tw_fwd + a.tw_off[ps], ps, P.q);
      __syncthreads();
    }
  } else {
    for (int ps = a.npass - 1; ps >= 1; --ps) {
      block_run_pass<false, NT, MAXEPI>(a, lds, P.tw_inv + a.tw_off[ps], ps, P.q);
      __syncthreads();
    }
  }
  for (int idx = threadIdx.x; idx < total; idx += NT) {
    const int t = idx >> glog, e = (idx & ((1 << glog) - 1)) * V;
    if (e0 + e < a.E)
      *(Vec<uint32_t, V>*)(buf + (size_t)t * a.E + e0 + e) =
          *(const Vec<uint32_t, V>*)(lds + t * pitch + e);
  }
}

// ---- register-resident block tile ------------------------------------------
// The same block step with the tile in registers: each of the NT threads
// holds PT positions (8, or 16 when a pass has 4 stages) of ET = 32 / PT
// adjacent entries, so a tile is NT * 32 residues (2^blk_log positions times
// 2^eb_log entries).  In a pass of r stages at stride S a thread runs PT / 2^r
// radix-2^r groups on its own registers; between passes the tile moves
// through LDS once (a write in one pass's position order, a read in the
// next's).  The first pass takes its values straight from the loads and the
// last one stores straight from registers, so LDS sees two accesses per
// residue per pass boundary and none at the ends.  Positions are swizzled in
// LDS so that the strided position sets of a wave spread over the banks.
// With 8 positions per thread: p ^ ((p >> 3) & 7) (no conflicts measured).
// With 16: bit b (b < 3) of p is xored with the parity of p & M_b,
// M_0 = 1658, M_1 = 1388, M_2 = 2800 (M_b holds no bit at or below b, so
// the map is a bijection on every aligned block of 8 or more positions);
// the masks came from a search over such maps against a model of the tile's
// LDS accesses that reproduced the measured conflict counts (32 banks, a
// wave's 8-byte accesses served 128 bytes at a time), and removed the 3
// conflict cycles per LDS instruction that the first map left in the
// {4,3,3} structures (measured at L = 2^14; no time change there, the LDS
// exchange being hidden).  Both maps are linear over GF(2), and a thread's
// position is the bitwise or of a part from its thread index and a part
// from its register index (disjoint bit fields), so the swizzle of the
// register part is a compile-time constant and the thread part's is
// computed once per pass.

template <int PT>
__host__ __device__ constexpr int reg_swz(int p) {
  if (PT == 8) return p ^ ((p >> 3) & 7);
  const unsigned x = (unsigned)p;
  return p ^ ((__builtin_popcount(x & 1658u) & 1) | ((__builtin_popcount(x & 1388u) & 1) << 1) |
              ((__builtin_popcount(x & 2800u) & 1) << 2));
}

// r stages at stride 2^s on each of the thread's PT / 2^r groups, twiddles
// of group c at tw[k S + j].  At stride 1 (s = 0) every group has j = 0, so
// its twiddles are the same for all lanes and those of w^0 = 1 are skipped.
template <bool DIF, int PT, int ET, int r, int s, bool LAZY>
__device__ __forceinline__ void reg_pass(uint32_t (&x)[ET][PT], int w,
                                         const Tw* __restrict__ tw, uint32_t q) {
  constexpr int R = 1 << r, S = 1 << s;
#pragma unroll
  for (int c = 0; c < PT / R; ++c) {
    const int wg = w * (PT / R) + c;
    const int j = wg & (S - 1);
    Tw t[R - 1];
#pragma unroll
    for (int k = 0; k < R - 1; ++k) t[k] = tw[k * S + j];
#pragma unroll
    for (int e = 0; e < ET; ++e) butterflies<r, DIF, false, s == 0, LAZY>(&x[e][c * R], t, q);
  }
}

// Whether a launch's block step fits the register tile with NT threads and
// PT positions per thread (the host picks the kernel with this).
__host__ __device__ inline bool reg_tile_fits(const NttLaunch& a, int nt_log, int pt_log) {
  if (!a.split || a.npass < 2) return false;
  int maxr = 0;
  for (int ps = 1; ps < a.npass; ++ps) maxr = a.stages[ps] > maxr ? a.stages[ps] : maxr;
  const int et_log = 5 - pt_log;
  return maxr <= pt_log && (pt_log == 4) == (maxr == 4) &&
         a.blk_log + a.eb_log == nt_log + 5 && a.eb_log >= et_log &&
         a.blk_log >= pt_log && a.vec >= (1 << et_log) && a.blk_pitch == (1 << a.eb_log);
}

// The register tile with the block passes fixed at compile time: R1, R2, R3
// stages in forward (decreasing-stride) order (R3 = 0: two passes), so all
// position and twiddle index arithmetic is shifts of constants.
template <int R1, int R2, int R3>
struct RegPasses {
  static constexpr int np = R3 ? 3 : 2;
  static constexpr int r(int i) { return i == 0 ? R1 : i == 1 ? R2 : R3; }
  static constexpr int s(int i) { return i == 0 ? R2 + R3 : i == 1 ? R3 : 0; }
};

template <int PT, int r, int s>
__host__ __device__ constexpr int reg_pos_c(int w, int v) {
  const int c = v >> r, u = v & ((1 << r) - 1);
  const int wg = w * (PT >> r) + c;
  return ((wg >> s) << (s + r)) + (wg & ((1 << s) - 1)) + (u << s);
}

template <bool DIF, int PT, int ET, int EBL, class RP, int K, bool LAZY>
__device__ __forceinline__ void reg_steps(uint32_t (&x)[ET][PT], int w, int el, uint32_t* lds,
                                          const uint32_t* twoff, const Tw* twb, uint32_t q,
                                          uint32_t* out, size_t E, bool live) {
  constexpr int i = DIF ? K : RP::np - 1 - K;           // pass in forward order
  constexpr int r = RP::r(i), s = RP::s(i);
  if constexpr (K > 0) {
    constexpr int ip = DIF ? K - 1 : RP::np - K;        // previous pass
    constexpr int rp = RP::r(ip), sp = RP::s(ip);
    // swizzled position = thread part ^ register part (see reg_swz)
    const int wp = reg_swz<PT>(reg_pos_c<PT, rp, sp>(w, 0));
    const int wc = reg_swz<PT>(reg_pos_c<PT, r, s>(w, 0));
#pragma unroll
    for (int v = 0; v < PT; ++v) {
      Vec<uint32_t, ET> y;
#pragma unroll
      for (int e = 0; e < ET; ++e) y.v[e] = x[e][v];
      const int sv = reg_swz<PT>(reg_pos_c<PT, rp, sp>(0, v));
      *(Vec<uint32_t, ET>*)(lds + ((wp ^ sv) << EBL) + el) = y;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < PT; ++v) {
      const int sv = reg_swz<PT>(reg_pos_c<PT, r, s>(0, v));
      const Vec<uint32_t, ET> y =
          *(const Vec<uint32_t, ET>*)(lds + ((wc ^ sv) << EBL) + el);
#pragma unroll
      for (int e = 0; e < ET; ++e) x[e][v] = y.v[e];
    }
    __syncthreads();
  }
  reg_pass<DIF, PT, ET, r, s, LAZY>(x, w, twb + twoff[i + 1], q);
  if constexpr (K + 1 < RP::np) {
    reg_steps<DIF, PT, ET, EBL, RP, K + 1, LAZY>(x, w, el, lds, twoff, twb, q, out, E, live);
  } else if (live) {
#pragma unroll
    for (int v = 0; v < PT; ++v) {
      Vec<uint32_t, ET> y;
#pragma unroll
      for (int e = 0; e < ET; ++e) y.v[e] = x[e][v];
      *(Vec<uint32_t, ET>*)(out + (size_t)reg_pos_c<PT, r, s>(w, v) * E) = y;
    }
  }
}

// EBL = eb_log: 2^EBL entries per tile (so NT * 32 = 2^(R1+R2+R3+EBL)).
template <bool DIF, int NT, int PT, int R1, int R2, int R3, bool LAZY>
__device__ __forceinline__ void block_tile_regc_t(const NttLaunch& a, int prime, int eb, int z,
                                                  uint32_t* lds) {
  using RP = RegPasses<R1, R2, R3>;
  constexpr int ET = 32 / PT;
  constexpr int BL = R1 + R2 + R3;                        // blk_log
  constexpr int EBL = (NT == 256 ? 13 : 14) - BL;         // eb_log
  constexpr int GL = EBL - (ET == 4 ? 2 : 1);
  const PrimeConst& P = a.pc[prime];
  const int g = threadIdx.x & ((1 << GL) - 1), w = threadIdx.x >> GL;
  const int el = g * ET;
  const bool live = (eb << EBL) + el < a.E;
  uint32_t* buf = (uint32_t*)a.out + a.out_prime_stride * prime + ((size_t)z << BL) * a.E +
                  ((size_t)eb << EBL) + el;
  constexpr int i0 = DIF ? 0 : RP::np - 1;
  uint32_t x[ET][PT];
#pragma unroll
  for (int v = 0; v < PT; ++v) {
    Vec<uint32_t, ET> y;
    if (live) {
      y = *(const Vec<uint32_t, ET>*)(buf + (size_t)reg_pos_c<PT, RP::r(i0), RP::s(i0)>(w, v) * a.E);
    } else {
#pragma unroll
      for (int e = 0; e < ET; ++e) y.v[e] = 0;
    }
#pragma unroll
    for (int e = 0; e < ET; ++e) x[e][v] = y.v[e];
  }
  reg_steps<DIF, PT, ET, EBL, RP, 0, LAZY>(x, w, el, lds, a.tw_off, DIF ? P.tw_fwd : P.tw_inv,
                                           P.q, buf, (size_t)a.E, live);
}

// The register tile, with lazy butterflies where the launch allows them
// (a.lazy: every residue it stores may lie in [0, 2q); the consumers accept
// that: the pointwise kernels, and the inverse's last pass, which reduces
// its inputs first).
template <bool DIF, int NT, int PT, int R1, int R2, int R3>
__device__ __forceinline__ void block_tile_regc(const NttLaunch& a, int prime, int eb, int z,
                                                uint32_t* lds) {
  if (a.lazy) block_tile_regc_t<DIF, NT, PT, R1, R2, R3, true>(a, prime, eb, z, lds);
  else block_tile_regc_t<DIF, NT, PT, R1, R2, R3, false>(a, prime, eb, z, lds);
}

// Register-tile kind of a launch's block step for 2^nt_log threads (0: the
// tile does not fit, or the passes are none of the compiled structures).
__host__ __device__ inline int reg_kind_of(const NttLaunch& a, int nt_log) {
  if (a.npass < 3 || a.npass > 4) return 0;
  const int r1 = a.stages[1], r2 = a.stages[2], r3 = a.npass == 4 ? a.stages[3] : 0;
  if (a.stride_log[1] != r2 + r3 || a.stride_log[2] != r3 || (r3 && a.stride_log[3] != 0))
    return 0;
  int kind = 0, pt_log = 4;
  if (r1 == 3 && r2 == 3 && r3 == 3) kind = 1, pt_log = 3;
  else if (r1 == 4 && r2 == 3 && r3 == 0) kind = 2;
  else if (r1 == 4 && r2 == 4 && r3 == 0) kind = 3;
  else if (r1 == 4 && r2 == 3 && r3 == 3) kind = 4;
  else if (r1 == 4 && r2 == 4 && r3 == 3) kind = 5;
  return kind && reg_tile_fits(a, nt_log, pt_log) ? kind : 0;
}

// The block step of a launch whose reg_kind is set, with NT threads.
template <bool DIF, int NT>
__device__ __forceinline__ void block_tile_reg_kind(const NttLaunch& a, int prime, int eb, int z,
                                                    uint32_t* lds) {
  switch (a.reg_kind) {
    case 1: block_tile_regc<DIF, NT, 8, 3, 3, 3>(a, prime, eb, z, lds); break;
    case 2: block_tile_regc<DIF, NT, 16, 4, 3, 0>(a, prime, eb, z, lds); break;
    case 3: block_tile_regc<DIF, NT, 16, 4, 4, 0>(a, prime, eb, z, lds); break;
    case 4: block_tile_regc<DIF, NT, 16, 4, 3, 3>(a, prime, eb, z, lds); break;
    default: block_tile_regc<DIF, NT, 16, 4, 4, 3>(a, prime, eb, z, lds); break;
  }
}

// First forward pass of a split transform, r stages at stride S = L / 2^r,
// items [it0, it1) with stride `step`: item (j, g) reads, for the CV entries
// e = g CV .. g CV + CV - 1, the rows j + u S below nin of the
// coefficient-major input and writes rows j + u S, u < keep, of the
// point-major buffer (keep = 2^r, or 3 2^r / 4 for a three-quarter
// transform: the last quarter of the rows feeds only the points dropped).
// ZHI (nin <= L/2): rows u >= 2^(r-1) are zero padding, not read, and the
// first stage reduces to products by the twiddles.  The entries share the
// twiddles.
template <typename TIn, bool REDUCE, int r, int CV, bool ZHI = true>
__device__ __forceinline__ void col_fwd_items(const NttLaunch& a, int prime, uint32_t it0,
                                              uint32_t it1, uint32_t step) {
  constexpr int R = 1 << r;
  const PrimeConst& P = a.pc[prime];
  const uint32_t q = P.q;
  const uint32_t S = 1u << (a.logL - r);
  const uint32_t E = (uint32_t)a.E, G = E / CV;
  const TIn* in = (const TIn*)a.in + a.in_prime_stride * prime;
  uint32_t* out = (uint32_t*)a.out + a.out_prime_stride * prime;
  const Tw* tw = P.tw_fwd + a.tw_off[0];
  const int keep = a.keep;
  for (uint32_t it = it0; it < it1; it += step) {
    const uint32_t j = it / G, e = (it - j * G) * CV;
    uint32_t x[CV][R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const uint32_t row = j + u * S;
      Vec<TIn, CV> v;
#pragma unroll
      for (int c = 0; c < CV; ++c) v.v[c] = 0;
      if ((!ZHI || u < R / 2) && row < (uint32_t)a.nin)
        v = load_nt((const Vec<TIn, CV>*)(in + (size_t)row * E + e));
#pragma unroll
      for (int c = 0; c < CV; ++c)
        x[c][u] = REDUCE ? reduce_u64((uint64_t)v.v[c], q, P.mu) : (uint32_t)v.v[c];
    }
    Tw t[R - 1];
#pragma unroll
    for (int k = 0; k < R - 1; ++k) t[k] = tw[k * S + j];
#pragma unroll
    for (int c = 0; c < CV; ++c) butterflies<r, true, ZHI>(x[c], t, q);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (u >= 3 * R / 4 && u >= keep) break;
      Vec<uint32_t, CV> y;
#pragma unroll
      for (int c = 0; c < CV; ++c) y.v[c] = x[c][u];
      *(Vec<uint32_t, CV>*)(out + (size_t)(j + u * S) * E + e) = y;
    }
  }
}

// CRT mode: the first pass of every prime's transform from one read of the
// input rows.  Item (j, g) loads rows j + u S (u < 2^(r-1): the inputs fill
// at most L/2 rows) once, then for each prime reduces them, runs the pass
// and writes that prime's rows u < keep; the per-prime launch reads the
// same input once per prime.
template <typename TIn, int r, int CV>
__device__ __forceinline__ void col_fwd_items_mp(const NttLaunch& a, int nprimes, uint32_t it0,
                                                 uint32_t it1, uint32_t step) {
  constexpr int R = 1 << r, H = R / 2;
  const uint32_t S = 1u << (a.logL - r);
  const uint32_t E = (uint32_t)a.E, G = E / CV;
  const TIn* in = (const TIn*)a.in;
  const int keep = a.keep;
  for (uint32_t it = it0; it < it1; it += step) {
    const uint32_t j = it / G, e = (it - j * G) * CV;
    Vec<TIn, CV> v[H];
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const uint32_t row = j + u * S;
#pragma unroll
      for (int c = 0; c < CV; ++c) v[u].v[c] = 0;
      if (row < (uint32_t)a.nin) v[u] = load_nt((const Vec<TIn, CV>*)(in + (size_t)row * E + e));
    }
#pragma unroll 1
    for (int i = 0; i < nprimes; ++i) {
      const PrimeConst& P = a.pc[i];
      const uint32_t q = P.q;
      uint32_t x[CV][R];
#pragma unroll
      for (int u = 0; u < H; ++u)
#pragma unroll
        for (int c = 0; c < CV; ++c) x[c][u] = reduce_u64((uint64_t)v[u].v[c], q, P.mu);
      const Tw* tw = P.tw_fwd + a.tw_off[0];
      Tw t[R - 1];
#pragma unroll
      for (int k = 0; k < R - 1; ++k) t[k] = tw[k * S + j];
#pragma unroll
      for (int c = 0; c < CV; ++c) butterflies<r, true, true>(x[c], t, q);
      uint32_t* out = (uint32_t*)a.out + a.out_prime_stride * i;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        if (u >= 3 * R / 4 && u >= keep) break;
        Vec<uint32_t, CV> y;
#pragma unroll
        for (int c = 0; c < CV; ++c) y.v[c] = x[c][u];
        *(Vec<uint32_t, CV>*)(out + (size_t)(j + u * S) * E + e) = y;
      }
    }
  }
}

// Passes of 5 stages take at most 2 entries per item (32 residues each).
template <typename TIn, int r>
__device__ __forceinline__ void col_fwd_tile_mp(const NttLaunch& a, int nprimes, uint32_t it0,
                                                uint32_t it1, uint32_t step) {
  constexpr int CVMAX = sizeof(TIn) == 8 || r >= 5 ? 2 : 4;
  if (a.col_vec >= CVMAX) col_fwd_items_mp<TIn, r, CVMAX>(a, nprimes, it0, it1, step);
  else if (a.col_vec >= 2) col_fwd_items_mp<TIn, r, 2>(a, nprimes, it0, it1, step);
  else col_fwd_items_mp<TIn, r, 1>(a, nprimes, it0, it1, step);
}

template <typename TIn, bool REDUCE, int r>
__device__ __forceinline__ void col_fwd_tile(const NttLaunch& a, int prime, uint32_t it0,
                                             uint32_t it1, uint32_t step) {
  if (2 * a.nin > (1 << a.logL)) {  // inputs longer than L/2 (coefficient windows)
    col_fwd_items<TIn, REDUCE, r, 1, false>(a, prime, it0, it1, step);
    return;
  }
  if constexpr (r < 5) {
    if (a.col_vec == 4) {
      col_fwd_items<TIn, REDUCE, r, 4>(a, prime, it0, it1, step);
      return;
    }
  }
  if (a.col_vec >= 2) col_fwd_items<TIn, REDUCE, r, 2>(a, prime, it0, it1, step);
  else col_fwd_items<TIn, REDUCE, r, 1>(a, prime, it0, it1, step);
}

// Inverse of a three-quarter first pass (r >= 2 stages, R = 2^r, Q = R/4):
// the forward pass kept its outputs u < 3Q, and the coefficients
// X_u = c_{j+uS} are zero for u >= 3Q (the product has fewer than 3L/4).
// The stages below distance R/4 are undone on each kept quarter and the one
// at distance R/4 on the first half; then, with c = j + uS (u < Q) and
// I = w^(L/4),
//   x[u] = (X_u + X_{u+2Q}) / 2,  x[u+Q] = X_{u+Q} / 2,
//   x[u+2Q] = w^c (X_u - X_{u+2Q} + I X_{u+Q}) / 4,
// so X_{u+Q} = 2 x[u+Q] and X_u, X_{u+2Q} = x[u] +- (2 w^-c x[u+2Q] - I x[u+Q]),
// w^-c being the twiddle of the top stage.  (The input rows carry the factor
// 1/R that the full inverse pass cancels, so the results are the
// coefficients themselves, as there.)
template <int r>
__device__ __forceinline__ void butterflies_inv34(uint32_t* x, const Tw* t, uint32_t q,
                                                  uint32_t i4, uint32_t i4p) {
  constexpr int R = 1 << r, H = R / 2, Q = R / 4;
  const uint32_t nq = opaque_neg(q);
#pragma unroll
  for (int v = 0; v < r - 2; ++v) {
#pragma unroll
    for (int u = 0; u < 3 * Q; ++u) {
      if (u & (1 << v)) continue;
      const int u2 = u | (1 << v);
      const Tw tt = t[(1 << v) - 1 + (u & ((1 << v) - 1))];
      const uint32_t a0 = x[u], b0 = mul_shoup_nq(x[u2], tt.w, tt.wp, q, nq);
      x[u] = add_mod(a0, b0, q);
      x[u2] = sub_mod(a0, b0, q);
    }
  }
#pragma unroll
  for (int u = 0; u < Q; ++u) {
    const Tw tt = t[Q - 1 + u];
    const uint32_t a0 = x[u], b0 = mul_shoup_nq(x[u + Q], tt.w, tt.wp, q, nq);
    x[u] = add_mod(a0, b0, q);
    x[u + Q] = sub_mod(a0, b0, q);
  }
#pragma unroll
  for (int u = 0; u < Q; ++u) {
    const Tw tt = t[H - 1 + u];
    const uint32_t g = mul_shoup_nq(x[u + H], tt.w, tt.wp, q, nq);
    const uint32_t ib = mul_shoup_nq(x[u + Q], i4, i4p, q, nq);
    const uint32_t s = sub_mod(add_mod(g, g, q), ib, q);
    const uint32_t a0 = x[u];
    x[u] = add_mod(a0, s, q);
    x[u + H] = sub_mod(a0, s, q);
    x[u + Q] = add_mod(x[u + Q], x[u + Q], q);
  }
}

// Last inverse pass of a split transform: item (j, g) reads rows j + u S of
// the point-major buffer for CV consecutive entries and writes coefficients
// out_lo .. out_lo + nin - 1 to rows 0 .. nin - 1 of the coefficient-major
// output.  TR: a three-quarter transform (rows u < 3 2^r / 4 only).  LAZYIN:
// the inputs lie in [0, 2q) and are reduced once on loading.
template <typename TOut, int r, int CV, bool TR, bool LAZYIN>
__device__ __forceinline__ void col_inv_items_t(const NttLaunch& a, int prime, uint32_t it0,
                                                uint32_t it1, uint32_t step) {
  constexpr int R = 1 << r;
  constexpr int KEEP = TR ? 3 * R / 4 : R;
  const PrimeConst& P = a.pc[prime];
  const uint32_t S = 1u << (a.logL - r);
  const uint32_t E = (uint32_t)a.E, G = E / CV;
  const uint32_t* in = (const uint32_t*)a.in + a.in_prime_stride * prime;
  TOut* out = (TOut*)a.out + a.out_prime_stride * prime;
  const Tw* tw = P.tw_inv + a.tw_off[0];
  for (uint32_t it = it0; it < it1; it += step) {
    const uint32_t j = it / G, e = (it - j * G) * CV;
    uint32_t x[CV][R];
#pragma unroll
    for (int u = 0; u < KEEP; ++u) {
      const Vec<uint32_t, CV> v = *(const Vec<uint32_t, CV>*)(in + (size_t)(j + u * S) * E + e);
#pragma unroll
      for (int c = 0; c < CV; ++c) x[c][u] = LAZYIN ? reduce_once(v.v[c], P.q) : v.v[c];
    }
    Tw t[R - 1];
#pragma unroll
    for (int k = 0; k < R - 1; ++k) t[k] = tw[k * S + j];
#pragma unroll
    for (int c = 0; c < CV; ++c) {
      if (TR) butterflies_inv34<r>(x[c], t, P.q, P.i4, P.i4p);
      else butterflies<r, false, false>(x[c], t, P.q);
    }
#pragma unroll
    for (int u = 0; u < KEEP; ++u) {
      const uint32_t row = j + u * S - (uint32_t)a.out_lo;  // wraps above nin below out_lo
      if (row < (uint32_t)a.nin) {
        Vec<TOut, CV> y;
#pragma unroll
        for (int c = 0; c < CV; ++c) y.v[c] = (TOut)x[c][u];
        *(Vec<TOut, CV>*)(out + (size_t)row * E + e) = y;
      }
    }
  }
}

template <typename TOut, int r, int CV, bool TR = false>
__device__ __forceinline__ void col_inv_items(const NttLaunch& a, int prime, uint32_t it0,
                                              uint32_t it1, uint32_t step) {
  // the register-tile block step before this pass left residues in [0, 2q);
  // the flag is uniform, so the canonical case carries no reduction
  if (a.lazy && a.reg_kind) col_inv_items_t<TOut, r, CV, TR, true>(a, prime, it0, it1, step);
  else col_inv_items_t<TOut, r, CV, TR, false>(a, prime, it0, it1, step);
}

// f(integral_constant<int, U>) for U in the sequence, unrolled whatever the
// size of f's body (a loop's unroll pragma gives up on large bodies, and an
// unrolled loop is what keeps register arrays out of scratch memory).
template <int... U, typename F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, U...>, F&& f) {
  (f(std::integral_constant<int, U>{}), ...);
}

// Last inverse pass of all NP primes' transforms with the Chinese
// remaindering folded in (CRT mode): item (j, e) runs the pass on rows j + uS
// of each prime's evaluations (one entry per item) and writes the
// coefficients mod p, rebuilt from the NP residues in registers, straight to
// the output C[row][e] (c.out), so the residues never go through HBM.
// TR: a three-quarter transform.  LAZYIN: the inputs lie in [0, 2q) and are
// reduced once on loading.
template <typename TOut, int r, int NP, bool TR, bool LAZYIN>
__device__ __forceinline__ void col_inv_crt_items(const NttLaunch& a, const CrtLaunch& c,
                                                  uint32_t it0, uint32_t it1, uint32_t step) {
  constexpr int R = 1 << r;
  constexpr int KEEP = TR ? 3 * R / 4 : R;
  const uint32_t S = 1u << (a.logL - r);
  const uint32_t E = (uint32_t)a.E;
  const CrtConsts<NP> cc(c);
  TOut* out = (TOut*)c.out;
  for (uint32_t it = it0; it < it1; it += step) {
    const uint32_t j = it / E, e = it - j * E;
    // Garner digits, row by row, formed as each prime's pass completes, so
    // only one prime's residues are live beside the digits.  The scheduling
    // barrier keeps the next prime's loads from being hoisted over this
    // prime's work (which would hold every prime's residues at once).
    uint32_t y[NP][R];
    static_for(std::make_integer_sequence<int, NP>{}, [&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const PrimeConst& P = a.pc[i];
      const uint32_t* in = (const uint32_t*)a.in + a.in_prime_stride * i;
      uint32_t x[R];
#pragma unroll
      for (int u = 0; u < KEEP; ++u) {
        x[u] = in[(size_t)(j + u * S) * E + e];
        if (LAZYIN) x[u] = reduce_once(x[u], P.q);
      }
      const Tw* tw = P.tw_inv + a.tw_off[0];
      Tw t[R - 1];
#pragma unroll
      for (int k = 0; k < R - 1; ++k) t[k] = tw[k * S + j];
      if (TR) butterflies_inv34<r>(x, t, P.q, P.i4, P.i4p);
      else butterflies<r, false, false>(x, t, P.q);
      static_for(std::make_integer_sequence<int, KEEP>{}, [&](auto uc) {
        constexpr int u = decltype(uc)::value;
        uint32_t v = x[u];
#pragma unroll
        for (int jj = 0; jj < i; ++jj) v = cc.step(i, jj, v, y[jj][u]);
        y[i][u] = v;
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    static_for(std::make_integer_sequence<int, KEEP>{}, [&](auto uc) {
      constexpr int u = decltype(uc)::value;
      const uint32_t row = j + u * S - (uint32_t)a.out_lo;  // wraps above nin below out_lo
      if (row < (uint32_t)a.nin) {
        uint32_t yu[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) yu[i] = y[i][u];
        out[(size_t)row * E + e] = (TOut)cc.combine(yu);
      }
    });
  }
}

template <typename TOut, int r, bool TR>
__device__ __forceinline__ void col_inv_tile_t(const NttLaunch& a, int prime, uint32_t it0,
                                               uint32_t it1, uint32_t step) {
  if constexpr (r < 5) {
    if (a.col_vec == 4) {
      col_inv_items<TOut, r, 4, TR>(a, prime, it0, it1, step);
      return;
    }
  }
  if (a.col_vec >= 2) col_inv_items<TOut, r, 2, TR>(a, prime, it0, it1, step);
  else col_inv_items<TOut, r, 1, TR>(a, prime, it0, it1, step);
}

template <typename TOut, int r>
__device__ __forceinline__ void col_inv_tile(const NttLaunch& a, int prime, uint32_t it0,
                                             uint32_t it1, uint32_t step) {
  if (a.keep < (1 << r)) col_inv_tile_t<TOut, r, true>(a, prime, it0, it1, step);
  else col_inv_tile_t<TOut, r, false>(a, prime, it0, it1, step);
}

}  // namespace pm
