// pm_crt_dev.h -- Chinese remaindering for moduli that are not FFT primes.
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
#pragma once
#include "pm_arith.h"
#include "pm_kernels.h"

namespace pm {

// The constants of R primes known at compile time, read once (the loops over
// primes unroll).
template <int R>
struct CrtConsts {
  uint32_t q[R], mu32[R], inv[R][R], invp[R][R];
  uint64_t radix[R];
  uint64_t p, mu_p;
  double pinv;

  __device__ __forceinline__ explicit CrtConsts(const CrtLaunch& a) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      q[i] = a.q[i];
      mu32[i] = a.mu32[i];
      radix[i] = a.radix_mod_p[i];
#pragma unroll
      for (int j = 0; j < i; ++j) {
        inv[i][j] = a.inv[i][j];
        invp[i][j] = a.inv_p[i][j];
      }
    }
    p = a.p;
    mu_p = a.mu_p;
    pinv = a.pinv;
  }

  // One Garner step for prime i: (t - y_j) q_j^{-1} mod q_i.
  __device__ __forceinline__ uint32_t step(int i, int j, uint32_t t, uint32_t yj) const {
    // y_j < q_j < 2^31: Barrett with floor(2^32 / q_i) leaves [0, 2 q_i)
    const uint32_t r = reduce_once(yj - __umulhi(yj, mu32[i]) * q[i], q[i]);
    return mul_shoup(sub_mod(t, r, q[i]), inv[i][j], invp[i][j], q[i]);
  }

  // X mod p from v[i] = X mod q_i (0 <= X < prod q_i).
  __device__ __forceinline__ uint64_t value(const uint32_t (&v)[R]) const {
    uint32_t y[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      uint32_t t = v[i];
#pragma unroll
      for (int j = 0; j < i; ++j) t = step(i, j, t, y[j]);
      y[i] = t;
    }
    return combine(y);
  }

  // X mod p from its Garner digits y_i.
  __device__ __forceinline__ uint64_t combine(const uint32_t (&y)[R]) const {
    uint64_t acc = 0;
    if (p <= 0xFFFFFFFFull) {
      // y_i (prod_{j<i} q_j mod p) < 2^63: Barrett with floor((2^64-1)/p)
      // leaves [0, 3p)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const uint64_t x = (uint64_t)y[i] * radix[i];
        uint64_t r = x - __umul64hi(x, mu_p) * p;
        if (r >= p) r -= p;
        if (r >= p) r -= p;
        acc += r;
        if (acc >= p) acc -= p;
      }
    } else {
      // S = sum_i y_i R_i with R_i = prod_{j<i} q_j mod p < 2^62 and
      // y_i < 2^31 is below 8 2^93 = 2^96: accumulate it exactly in 96 bits
      // (lo: 64, hi: 32), then reduce once.  S / p < r 2^31 <= 2^34 (each
      // R_i < p), and S and 1/p carry relative rounding errors near 2^-53,
      // so the double-precision quotient estimate is within one of the true
      // quotient and the remainder computed mod 2^64 needs one signed
      // correction.
      uint64_t lo = 0;
      uint32_t hi = 0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const uint64_t pl = (uint64_t)y[i] * (uint32_t)radix[i];          // < 2^63
        const uint64_t ph = (uint64_t)y[i] * (uint32_t)(radix[i] >> 32);  // < 2^61
        const uint64_t t = lo + pl;
        hi += t < pl;
        const uint64_t sh = ph << 32;
        lo = t + sh;
        hi += (uint32_t)(ph >> 32) + (lo < sh);
      }
      const double sd = (double)hi * 18446744073709551616.0 + (double)lo;
      const uint64_t qt = (uint64_t)(sd * pinv);
      int64_t r = (int64_t)(lo - qt * p);  // exact mod 2^64, |r| < 2p < 2^63
      if (r < 0) r += (int64_t)p;
      if (r >= (int64_t)p) r -= (int64_t)p;
      acc = (uint64_t)r;
    }
    return acc;
  }
};

// Outputs idx = i0, i0 + step, ... below min(i1, count), for R primes known
// at compile time.
template <typename TOut, int R>
__device__ __forceinline__ void crt_range_r(const CrtLaunch& a, uint64_t i0, uint64_t i1,
                                            uint64_t step) {
  if (i1 > a.count) i1 = a.count;
  const CrtConsts<R> cc(a);
  const uint64_t pstride = a.prime_stride;
  for (uint64_t idx = i0; idx < i1; idx += step) {
    uint32_t v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = a.cq[pstride * i + idx];
    ((TOut*)a.out)[idx] = (TOut)cc.value(v);
  }
}

template <typename TOut>
__device__ __forceinline__ void crt_range(const CrtLaunch& a, uint64_t i0, uint64_t i1,
                                          uint64_t step) {
  switch (a.r) {
    case 1: crt_range_r<TOut, 1>(a, i0, i1, step); break;
    case 2: crt_range_r<TOut, 2>(a, i0, i1, step); break;
    case 3: crt_range_r<TOut, 3>(a, i0, i1, step); break;
    case 4: crt_range_r<TOut, 4>(a, i0, i1, step); break;
    case 5: crt_range_r<TOut, 5>(a, i0, i1, step); break;
    case 6: crt_range_r<TOut, 6>(a, i0, i1, step); break;
    case 7: crt_range_r<TOut, 7>(a, i0, i1, step); break;
    default: crt_range_r<TOut, 8>(a, i0, i1, step); break;
  }
}

}  // namespace pm
