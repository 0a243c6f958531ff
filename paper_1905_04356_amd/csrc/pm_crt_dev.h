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

// Outputs idx = i0, i0 + step, ... below min(i1, count).
template <typename TOut>
__device__ __forceinline__ void crt_range(const CrtLaunch& a, uint64_t i0, uint64_t i1,
                                          uint64_t step) {
  if (i1 > a.count) i1 = a.count;
  for (uint64_t idx = i0; idx < i1; idx += step) {
    uint32_t y[kMaxPrimes];
    for (int i = 0; i < a.r; ++i) {
      const uint32_t qi = a.q[i];
      uint32_t t = a.cq[a.prime_stride * i + idx];
      for (int j = 0; j < i; ++j) {
        // y_j < q_j < 2^31: Barrett with floor(2^32 / q_i) leaves [0, 2 q_i)
        const uint32_t yj = reduce_once(y[j] - __umulhi(y[j], a.mu32[i]) * qi, qi);
        t = sub_mod(t, yj, qi);
        t = mul_shoup(t, a.inv[i][j], a.inv_p[i][j], qi);
      }
      y[i] = t;
    }
    uint64_t acc = 0;
    if (a.p <= 0xFFFFFFFFull) {
      // y_i (prod_{j<i} q_j mod p) < 2^63: Barrett with floor((2^64-1)/p)
      // leaves [0, 3p)
      for (int i = 0; i < a.r; ++i) {
        const uint64_t x = (uint64_t)y[i] * a.radix_mod_p[i];
        uint64_t r = x - __umul64hi(x, a.mu_p) * a.p;
        if (r >= a.p) r -= a.p;
        if (r >= a.p) r -= a.p;
        acc += r;
        if (acc >= a.p) acc -= a.p;
      }
    } else {
      for (int i = 0; i < a.r; ++i) {
        acc += mulmod_u64_small(y[i], a.radix_mod_p[i], a.p, a.pinv);
        if (acc >= a.p) acc -= a.p;
      }
    }
    ((TOut*)a.out)[idx] = (TOut)acc;
  }
}

}  // namespace pm
