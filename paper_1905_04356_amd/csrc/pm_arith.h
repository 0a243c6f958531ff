// pm_arith.h -- word-size modular arithmetic for the gfx950 kernels.
//
// All moduli q used inside transforms are primes below 2^31, so every residue
// and every sum of two residues fits in 32 bits.  The published methods used:
//   * Shoup's multiplication by a precomputed constant (V. Shoup, NTL; also
//     D. Harvey, "Faster arithmetic for number-theoretic transforms", 2014):
//     for a fixed w < q store w' = floor(w * 2^32 / q); then for any a < 2^32
//     the value a*w - floor(a*w'/2^32)*q lies in [0, 2q).
//   * Barrett reduction (P. Barrett, CRYPTO 1986) of 64-bit values with
//     mu = floor((2^64-1)/q).
//   * A floating-point estimate of the quotient for a*b mod p with p < 2^62
//     (the idea behind NTL's word-size MulMod with a precomputed 1/p): when
//     a*b/p < 2^50 the rounded estimate is within one of the true quotient,
//     so the remainder computed mod 2^64 needs one signed correction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

// min(x, x - q) in unsigned arithmetic: maps [0, 2q) onto [0, q).
__device__ __forceinline__ uint32_t reduce_once(uint32_t x, uint32_t q) {
  uint32_t y = x - q;
  return y < x ? y : x;
}

// (a + b) mod q for a, b in [0, q).
__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t q) {
  return reduce_once(a + b, q);
}

// (a - b) mod q for a, b in [0, q): min(a - b, a - b + q) in unsigned
// arithmetic.  If a >= b the first is in [0, q) and the second is larger;
// otherwise the first wraps to at least 2^32 - q > q and the second is the
// residue in [1, q).
__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t q) {
  const uint32_t d = a - b;
  const uint32_t e = d + q;
  return e < d ? e : d;
}

// a*w mod q in [0, 2q) for any a < 2^32, w < q, wp = floor(w*2^32/q).
__device__ __forceinline__ uint32_t mul_shoup_lazy(uint32_t a, uint32_t w, uint32_t wp,
                                                   uint32_t q) {
  uint32_t qt = __umulhi(a, wp);
  return a * w - qt * q;
}

// a*w mod q in [0, q).
__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wp,
                                              uint32_t q) {
  return reduce_once(mul_shoup_lazy(a, w, wp, q), q);
}

// 2^32 - q, hidden from the optimizer (see mul_shoup_nq).
__device__ __forceinline__ uint32_t opaque_neg(uint32_t q) {
  uint32_t nq = 0u - q;
  asm("" : "+v"(nq));
  return nq;
}

// mul_shoup with nq = 2^32 - q: a*w - qt*q mod 2^32 is the low word of
// qt*nq + (a*w mod 2^32), one v_mad_u64_u32 in place of a multiply and a
// subtraction.  (With nq visible as 0 - q the compiler folds the product
// back into the multiply-and-subtract form.)
__device__ __forceinline__ uint32_t mul_shoup_nq(uint32_t a, uint32_t w, uint32_t wp,
                                                 uint32_t q, uint32_t nq) {
  const uint32_t qt = __umulhi(a, wp);
  return reduce_once((uint32_t)((uint64_t)qt * nq + (uint64_t)(a * w)), q);
}

// mul_shoup_nq without the final correction: a*w mod q in [0, 2q) for any
// a < 2^32 (Harvey's lazy range).
__device__ __forceinline__ uint32_t mul_shoup_lazy_nq(uint32_t a, uint32_t w, uint32_t wp,
                                                      uint32_t nq) {
  const uint32_t qt = __umulhi(a, wp);
  return (uint32_t)((uint64_t)qt * nq + (uint64_t)(a * w));
}

// x mod q for any 64-bit x; mu = floor((2^64-1)/q).
__device__ __forceinline__ uint32_t reduce_u64(uint64_t x, uint32_t q, uint64_t mu) {
  uint64_t qt = __umul64hi(x, mu);
  uint64_t r = x - qt * (uint64_t)q;  // in [0, 3q)
  if (r >= q) r -= q;
  if (r >= q) r -= q;
  return (uint32_t)r;
}

// a*b mod p for a < 2^32 and b < p < 2^62; pinv = 1.0 / p (rounded).
__device__ __forceinline__ uint64_t mulmod_u64_small(uint64_t a, uint64_t b, uint64_t p,
                                                     double pinv) {
  // a*b/p < a < 2^32, so the rounded quotient is off by at most one.
  uint64_t qt = (uint64_t)((double)a * (double)b * pinv);
  int64_t r = (int64_t)(a * b - qt * p);  // exact mod 2^64, |r| < 2p < 2^63
  if (r < 0) r += (int64_t)p;
  if (r >= (int64_t)p) r -= (int64_t)p;
  return (uint64_t)r;
}

}  // namespace pm
