// pm_vdm.hip -- matrix products over F_p on the matrix cores, for evaluation
// and interpolation by Vandermonde matrices.
//
// Hyun, Neiger, Schost (ISSAC 2019), Section 2, "Polynomial matrix
// multiplication": an adaptation of the integer algorithm of Doliskani,
// Giorgi, Lebreton and Schost evaluates and interpolates by plain
// multiplication with (inverse) Vandermonde matrices, so that for moderate
// degrees the work is matrix multiplication over F_p.  Here one kernel
// computes Z = X Y mod q for row-major X (M x K), Y (K x N) with q < 2^31: a
// workgroup owns a 64 x 64 tile of Z and walks K in chunks of 64; both
// operands are staged in LDS as four planes of balanced int8 digits (as in
// the pointwise kernel), each wave accumulates its 32 x 32 quadrant with
// v_mfma_i32_16x16x64_i8 into seven weight classes, and the epilogue
// recombines them with Montgomery's reduction.  |acc_s| <= 4 K 2^14, so the
// bias q 7 K 2^16 keeps the weighted sum in [0, q 2^32) for K <= 4096.
#include "pm_pointwise_dev.h"
#include "pm_vdm.h"
#include "pm_profile.h"

namespace pm {

namespace {

constexpr int kTM = 64, kTN = 64, kTK = 64, kRS = kTK + 16;

template <bool CENTER>
__device__ __forceinline__ void stage_x(const GemmLaunch& g, int i0, int k0,
                                        uint8_t (*Xs)[kTM][kRS]) {
  const uint32_t q = g.q, hq = g.q >> 1;
  for (int it = threadIdx.x; it < kTM * (kTK / 4); it += blockDim.x) {
    const int r = it >> 4, grp = it & 15;       // row, group of 4 k
    const int i = i0 + r, k = k0 + 4 * grp;
    uint32_t in[4], out[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t v = (i < g.M && k + c < g.K) ? g.X[(size_t)i * g.ldx + k + c] : 0u;
      in[c] = limbs_of<CENTER>(v, q, hq);
    }
    transpose4x4(in, out);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) *(uint32_t*)&Xs[pl][r][4 * grp] = out[pl];
  }
}

template <bool CENTER>
__device__ __forceinline__ void stage_y(const GemmLaunch& g, int k0, int j0,
                                        uint8_t (*Ys)[kTN][kRS]) {
  const uint32_t q = g.q, hq = g.q >> 1;
  for (int it = threadIdx.x; it < kTN * (kTK / 4); it += blockDim.x) {
    const int jj = it & 63, grp = it >> 6;      // column, group of 4 k
    const int j = j0 + jj, k = k0 + 4 * grp;
    uint32_t in[4], out[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t v = (j < g.N && k + c < g.K) ? g.Y[(size_t)(k + c) * g.ldy + j] : 0u;
      in[c] = limbs_of<CENTER>(v, q, hq);
    }
    transpose4x4(in, out);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) *(uint32_t*)&Ys[pl][jj][4 * grp] = out[pl];
  }
}

template <bool CENTER>
__global__ __launch_bounds__(256) void gemm_modp_kernel(GemmLaunch g) {
  __shared__ uint8_t Xs[4][kTM][kRS];
  __shared__ uint8_t Ys[4][kTN][kRS];
  const int i0 = blockIdx.y * kTM, j0 = blockIdx.x * kTN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qi = wave & 1, qj = wave >> 1;
  const int lr = lane & 15, lk = (lane >> 4) * 16;
  v4i acc[2][2][7];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int s = 0; s < 7; ++s) acc[a][b][s] = (v4i){0, 0, 0, 0};
  for (int k0 = 0; k0 < g.K; k0 += kTK) {
    stage_x<CENTER>(g, i0, k0, Xs);
    stage_y<CENTER>(g, k0, j0, Ys);
    __syncthreads();
    v4i av[2][4], bv[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        av[a][pl] = *(const v4i*)&Xs[pl][32 * qi + 16 * a + lr][lk];
        bv[a][pl] = *(const v4i*)&Ys[pl][32 * qj + 16 * a + lr][lk];
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y)
            acc[a][b][x + y] =
                __builtin_amdgcn_mfma_i32_16x16x64_i8(av[a][x], bv[b][y], acc[a][b][x + y], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = j0 + 32 * qj + 16 * b + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + 32 * qi + 16 * a + (lane >> 4) * 4 + r;
        int64_t S = (int64_t)g.bias;
#pragma unroll
        for (int s = 0; s < 7; ++s) S += (int64_t)(int32_t)g.cs[s] * (int64_t)acc[a][b][s][r];
        const uint32_t mm = (uint32_t)S * g.qninv;
        const uint32_t v = reduce_once((uint32_t)(((uint64_t)mm * g.q + (uint64_t)S) >> 32), g.q);
        if (i < g.M && j < g.N) g.Z[(size_t)i * g.ldz + j] = v;
      }
    }
}

}  // namespace

int launch_gemm_modp(const GemmLaunch& g, hipStream_t s) {
  if (g.M < 1 || g.N < 1 || g.K < 1 || g.K > kGemmMaxK || g.q >= (1u << 31))
    return hipErrorInvalidValue;
  const dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM);
  if (g.q <= 0x7F7F7F7Fu)
    return launch(gemm_modp_kernel<false>, grid, dim3(256), 0, s, g);
  else
    return launch(gemm_modp_kernel<true>, grid, dim3(256), 0, s, g);
}

}  // namespace pm
