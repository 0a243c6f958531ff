// pm_vdm.h -- matrix products over F_p on the matrix cores (Vandermonde
// evaluation and interpolation); see pm_vdm.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

constexpr int kGemmMaxK = 4096;  // keeps the Montgomery sum below q 2^32

// Z = X Y mod q: X row-major M x K (leading dimension ldx), Y row-major
// K x N (ldy), Z row-major M x N (ldz); q odd, q < 2^31; entries of X and
// Y in [0, q).  cs[s] = 256^s 2^32 mod q, bias = q 7 K 2^16,
// qninv = -q^{-1} mod 2^32.
struct GemmLaunch {
  int M, N, K;
  int ldx, ldy, ldz;
  const uint32_t* X;
  const uint32_t* Y;
  uint32_t* Z;
  uint32_t q;
  uint32_t qninv;
  uint32_t cs[8];
  uint64_t bias;
};

int launch_gemm_modp(const GemmLaunch& g, hipStream_t s);

}  // namespace pm
