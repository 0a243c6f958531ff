// pm_pointwise_dev.h -- device side of the matrix products at the evaluation points.
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
#pragma once
#include "pm_arith.h"
#include "pm_kernels.h"

namespace pm {

template <bool STAGED>
__device__ __forceinline__ void pointwise_valu_tile(const PointwiseLaunch& a, int t, int prime,
                                                    uint32_t* sm) {
  const PrimeConst& P = a.pc[prime];
  const uint32_t q = P.q;
  const size_t mn = (size_t)a.m * a.n, nk = (size_t)a.n * a.k, mk = (size_t)a.m * a.k;
  const uint32_t* A = a.ahat + a.a_prime_stride * prime + (size_t)t * mn;
  const uint32_t* B = a.bhat + a.b_prime_stride * prime + (size_t)t * nk;
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

// ---- int8-MFMA variant ---------------------------------------------------------
//
// Exact products on the matrix cores.  A residue x in [0, q) is centred,
// x' = x - q if x > q/2, so |x'| < 2^30, and written with four balanced
// base-256 digits x' = sum_a x_a 256^a, x_a in [-128, 127]: adding
// 0x80808080 turns x' into an unsigned word whose bytes are x_a + 128, so
// (x' + 0x80808080) ^ 0x80808080 holds the four int8 digits.  Then
//   A_t B_t = sum_{s=0..6} 256^s acc_s,   acc_s = sum_{a+b=s} A_a B_b,
// 16 int8 GEMMs with int32 accumulation (|acc_s| <= 4 n 2^14 < 2^31 for
// n < 2^15), recombined as sum_s c_s acc_s mod q in int64 with
// c_s = 256^s L^{-1} mod q (|sum| < n 2^49, exact while n < 2^13).
//
// One workgroup (4 or 8 waves) per point: the two matrices are loaded with
// coalesced 16-byte reads, split, and stored as limb planes in LDS
// (A: plane, row i, contraction index l; B transposed: plane, column j, l);
// each wave then computes 16x16 output tiles with v_mfma_i32_16x16x64_i8.
// Contractions of at most 16 are packed (see kK16Row), and large limb
// planes run the pipelined variant at the end of this file, where a
// workgroup runs a sequence of points.
// Lane layout of that instruction (checked on gfx950): lane L supplies
// A[L%16][16(L/16) + b] and B[16(L/16) + b][L%16] for bytes b < 16, and
// receives C[4(L/16) + r][L%16] for r < 4.

typedef int v4i __attribute__((ext_vector_type(4)));

// Byte-transpose of four words: out[a] byte c = in[c] byte a.
__device__ __forceinline__ void transpose4x4(const uint32_t in[4], uint32_t out[4]) {
  // v_perm_b32(hi, lo, sel): selector bytes 0-3 pick from lo, 4-7 from hi.
  const uint32_t t0 = __builtin_amdgcn_perm(in[1], in[0], 0x05010400u);  // in0.0 in1.0 in0.1 in1.1
  const uint32_t t1 = __builtin_amdgcn_perm(in[1], in[0], 0x07030602u);  // in0.2 in1.2 in0.3 in1.3
  const uint32_t t2 = __builtin_amdgcn_perm(in[3], in[2], 0x05010400u);
  const uint32_t t3 = __builtin_amdgcn_perm(in[3], in[2], 0x07030602u);
  out[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);  // t0.0 t0.1 t2.0 t2.1
  out[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);  // t0.2 t0.3 t2.2 t2.3
  out[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
  out[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// Four balanced base-256 digits (each in [-128, 127]) of x as bytes: the sum
// x + 0x80808080 carries exactly as the balanced representation needs, and
// the xor recentres each byte.  Exact for x in [-0x80808080, 0x7F7F7F7F] as a
// two's-complement word.  Residues below q <= 0x7F7F7F7F (all NTT primes
// used here) need no centring; larger q are centred first.
template <bool CENTER>
__device__ __forceinline__ uint32_t limbs_of(uint32_t x, uint32_t q, uint32_t half_q) {
  const uint32_t c = CENTER && x > half_q ? x - q : x;
  return (c + 0x80808080u) ^ 0x80808080u;
}

// A (row-major m x n) and B (n x k, stored transposed) into LDS digit planes.
template <bool CENTER>
__device__ __forceinline__ void stage_limbs(const uint32_t* A, const uint32_t* B, uint8_t* As,
                                            uint8_t* Bs, int m, int n, int k, int mp, int kp,
                                            int ng, int rs, uint32_t q, uint32_t half_q) {
  const int l16 = threadIdx.x & 15, r16 = threadIdx.x >> 4, nr = blockDim.x >> 4;
  // A: row i, 4 consecutive l per item; 16 lanes cover 64 consecutive l.
  for (int i = r16; i < mp; i += nr) {
    for (int g = l16; g < ng; g += 16) {
      const int l0 = g * 4;
      uint32_t in[4] = {0, 0, 0, 0}, out[4];
      if (i < m && l0 < n) {
        const uint4 v = *(const uint4*)(A + i * n + l0);
        in[0] = limbs_of<CENTER>(v.x, q, half_q); in[1] = limbs_of<CENTER>(v.y, q, half_q);
        in[2] = limbs_of<CENTER>(v.z, q, half_q); in[3] = limbs_of<CENTER>(v.w, q, half_q);
      }
      transpose4x4(in, out);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) *(uint32_t*)(As + (pl * mp + i) * rs + l0) = out[pl];
    }
  }
  // B transposed: column j, 4 consecutive l; 16 lanes cover 16 consecutive j.
  for (int g = r16; g < ng; g += nr) {
    const int l0 = g * 4;
    for (int j = l16; j < kp; j += 16) {
      uint32_t in[4] = {0, 0, 0, 0}, out[4];
      if (j < k && l0 < n) {
#pragma unroll
        for (int c = 0; c < 4; ++c) in[c] = limbs_of<CENTER>(B[(l0 + c) * k + j], q, half_q);
      }
      transpose4x4(in, out);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) *(uint32_t*)(Bs + (pl * kp + j) * rs + l0) = out[pl];
    }
  }
}

// Contractions of at most 16 (n <= 16) are packed instead of padded to 64:
// the four limb planes of A fill the 64 contraction bytes of one
// v_mfma_i32_16x16x64_i8 (lanes 16g .. 16g + 15 supply plane g of A's row),
// and for weight class s the same lanes supply plane s - g of B's column (a
// zero row where s - g is outside 0 .. 3), so one instruction sums A_a B_b
// over a + b = s: 7 instructions per output tile instead of 16, on LDS rows
// of 16 bytes.
constexpr int kK16Row = 16;

// The products of point t from the limb planes in LDS: 16x16 output tiles
// spread over the workgroup's waves, recombined, reduced and stored.  K16:
// the packed form (rows of kK16Row bytes, B's zero row after its planes).
template <bool K16 = false>
__device__ __forceinline__ void mfma_point(const PointwiseLaunch& a, int t, int prime,
                                           const uint8_t* As, const uint8_t* Bs, int mp, int kp,
                                           int np, int rs) {
  const PrimeConst& P = a.pc[prime];
  const uint32_t q = P.q;
  const int m = a.m, k = a.k;
  uint32_t* C = a.chat + a.prime_stride * prime + (size_t)t * ((size_t)m * k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int tiles_m = mp >> 4, tiles = tiles_m * (kp >> 4);
  const int lr = lane & 15, lk = (lane >> 4) * 16;
  // c_s < q < 2^31, so each weight is a non-negative int32 and each term a
  // single signed 32x32->64 multiply-add.  The bias, a multiple of q above
  // every |sum|, makes the sum T non-negative and T < 14 q n 2^16 <= q 2^32
  // (n < 4096), so Montgomery's reduction (P. Montgomery, Math. Comp. 1985)
  // t = (T + (T mu' mod 2^32) q) / 2^32 lies in [0, 2q) and equals
  // T 2^{-32} mod q; the weights carry the factor 2^32.
  int32_t cs[7];
#pragma unroll
  for (int s = 0; s < 7; ++s) cs[s] = (int32_t)a.cs[prime][s];
  const uint64_t bias = a.bias[prime];
  const uint32_t qninv = a.qninv[prime];
  for (int tile = wave; tile < tiles; tile += nwaves) {
    const int ti = tile % tiles_m, tj = tile / tiles_m;
    v4i acc[7];
#pragma unroll
    for (int s = 0; s < 7; ++s) acc[s] = (v4i){0, 0, 0, 0};
    if (K16) {
      const int g = lane >> 4;
      const v4i av = *(const v4i*)(As + (g * mp + ti * 16 + lr) * kK16Row);
      const uint8_t* zero = Bs + 4 * kp * kK16Row;
#pragma unroll
      for (int s = 0; s < 7; ++s) {
        const int x = s - g;
        const uint8_t* src = x >= 0 && x < 4 ? Bs + (x * kp + tj * 16 + lr) * kK16Row : zero;
        acc[s] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, *(const v4i*)src, acc[s], 0, 0, 0);
      }
    }
    for (int kc = 0; kc < (K16 ? 0 : np); kc += 64) {
      v4i av[4], bv[4];
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        av[pl] = *(const v4i*)(As + (pl * mp + ti * 16 + lr) * rs + kc + lk);
        bv[pl] = *(const v4i*)(Bs + (pl * kp + tj * 16 + lr) * rs + kc + lk);
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x + y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[x], bv[y], acc[x + y], 0, 0, 0);
    }
    const int j = tj * 16 + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = ti * 16 + (lane >> 4) * 4 + r;
      int64_t S = (int64_t)bias;
#pragma unroll
      for (int s = 0; s < 7; ++s) S += (int64_t)cs[s] * (int64_t)acc[s][r];
      const uint32_t mm = (uint32_t)S * qninv;
      const uint32_t v = reduce_once((uint32_t)(((uint64_t)mm * q + (uint64_t)S) >> 32), q);
      if (i < m && j < k) C[i * k + j] = v;
    }
  }
}

// A (m x n, n <= 16, a multiple of 4) and B (n x k, stored transposed) into
// packed limb planes: A plane a row i and B plane b column j are 16-byte
// rows (contraction indices 0 .. 15, zeros from n on); then B's zero row.
template <bool CENTER>
__device__ __forceinline__ void stage_limbs_k16(const uint32_t* A, const uint32_t* B,
                                                uint8_t* As, uint8_t* Bs, int m, int n, int k,
                                                int mp, int kp, uint32_t q, uint32_t half_q) {
  const int nt = blockDim.x;
  // A: item f = 4 i + g, the 16-byte group g of row i
  for (int f = threadIdx.x; f < 4 * mp; f += nt) {
    const int i = f >> 2, l0 = (f & 3) * 4;
    uint32_t in[4] = {0, 0, 0, 0}, out[4];
    if (i < m && l0 < n) {
      const uint4 v = *(const uint4*)(A + i * n + l0);
      in[0] = limbs_of<CENTER>(v.x, q, half_q); in[1] = limbs_of<CENTER>(v.y, q, half_q);
      in[2] = limbs_of<CENTER>(v.z, q, half_q); in[3] = limbs_of<CENTER>(v.w, q, half_q);
    }
    transpose4x4(in, out);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) *(uint32_t*)(As + (pl * mp + i) * kK16Row + l0) = out[pl];
  }
  // B: item f = g kp + j, rows 4g .. 4g + 3 of column j (consecutive threads,
  // consecutive columns)
  for (int f = threadIdx.x; f < 4 * kp; f += nt) {
    const int g = f / kp, j = f - g * kp, l0 = g * 4;
    uint32_t in[4] = {0, 0, 0, 0}, out[4];
    if (j < k && l0 < n) {
#pragma unroll
      for (int c = 0; c < 4; ++c) in[c] = limbs_of<CENTER>(B[(l0 + c) * k + j], q, half_q);
    }
    transpose4x4(in, out);
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) *(uint32_t*)(Bs + (pl * kp + j) * kK16Row + l0) = out[pl];
  }
  if (threadIdx.x < kK16Row / 4) ((uint32_t*)(Bs + 4 * kp * kK16Row))[threadIdx.x] = 0u;
}

__device__ __forceinline__ void pointwise_mfma_tile(const PointwiseLaunch& a, int t, int prime,
                                                    uint32_t* smem) {
  const PrimeConst& P = a.pc[prime];
  const uint32_t q = P.q, half_q = P.q >> 1;
  const int m = a.m, n = a.n, k = a.k;
  const int mp = (m + 15) & ~15, kp = (k + 15) & ~15, np = (n + 63) & ~63;
  if (n <= 16) {
    uint8_t* As = (uint8_t*)smem;             // [4][mp][16]
    uint8_t* Bs = As + 4 * mp * kK16Row;      // [4][kp][16], then 16 zero bytes
    const uint32_t* A = a.ahat + a.a_prime_stride * prime + (size_t)t * ((size_t)m * n);
    const uint32_t* B = a.bhat + a.b_prime_stride * prime + (size_t)t * ((size_t)n * k);
    if (q <= 0x7F7F7F7Fu)
      stage_limbs_k16<false>(A, B, As, Bs, m, n, k, mp, kp, q, half_q);
    else
      stage_limbs_k16<true>(A, B, As, Bs, m, n, k, mp, kp, q, half_q);
    __syncthreads();
    mfma_point<true>(a, t, prime, As, Bs, mp, kp, kK16Row, kK16Row);
    return;
  }
  const int rs = np + 16;                   // bytes per LDS row (padded)
  uint8_t* As = (uint8_t*)smem;             // [4][mp][rs]
  uint8_t* Bs = As + 4 * mp * rs;           // [4][kp][rs]
  const uint32_t* A = a.ahat + a.a_prime_stride * prime + (size_t)t * ((size_t)m * n);
  const uint32_t* B = a.bhat + a.b_prime_stride * prime + (size_t)t * ((size_t)n * k);
  const int ng = np >> 2;                   // groups of 4 contraction indices (multiple of 16)
  if (q <= 0x7F7F7F7Fu)
    stage_limbs<false>(A, B, As, Bs, m, n, k, mp, kp, ng, rs, q, half_q);
  else
    stage_limbs<true>(A, B, As, Bs, m, n, k, mp, kp, ng, rs, q, half_q);
  __syncthreads();
  mfma_point(a, t, prime, As, Bs, mp, kp, np, rs);
}

// ---- pipelined int8-MFMA variant --------------------------------------------
//
// Where the limb planes leave only one to three workgroups on a CU, a
// workgroup that loads, converts, multiplies and stores one point after the
// other leaves HBM idle while its matrix cores work.  Here a workgroup runs
// a sequence of points and the residues of the next point are already on
// their way into registers while the matrix cores work on this one.  Each
// thread owns the same items at every point: up to PA 16-byte groups of A
// (row i, contraction indices 4g .. 4g + 3; consecutive threads take
// consecutive groups of a row) and up to PB 4 x 4 blocks of B (rows
// 4g .. 4g + 3, columns 4h .. 4h + 3, one 16-byte load per row; 16
// consecutive threads take consecutive g, and 4 such groups consecutive h,
// so that a wave reads 64-byte runs of 16 rows and its transposed LDS
// stores hit 64 distinct banks).  B's row length k must be a multiple of 4.
// The barriers between the phases order only LDS accesses, so they do not
// wait for those loads.

// Barrier for the workgroup's LDS accesses only; global loads in flight stay
// in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// x, hidden from the optimiser: the slot coordinates derived from it are
// recomputed at each point instead of being kept live across the loop in
// registers (a handful of ALU operations against 2-4 registers per slot).
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// One point's items of this thread in registers.
template <int PA, int PB>
struct PipeRegs {
  uint4 a[PA];
  uint4 b[PB][4];
};

// Item coordinates.  A item f = i ng + g; B item f = 64 (hh G16 + gh) + 16 hl
// + gl with g = 16 gh + gl, h = 4 hh + hl (G16 = ng / 16).  The quotients
// take one high multiply: for divisors 2 <= D < 2^12, floor(f ceil(2^32 /
// D) / 2^32) = floor(f / D) as long as f D < 2^32 (here f < 2^13).  D = 1
// (G16 when ng = 16) has no 32-bit multiplier and is taken apart.
struct PipeShape {
  int m, n, k, mp, kp, ng, rs;
  uint32_t na, nb, g16, rng, rg16;
  __device__ __forceinline__ PipeShape(int m_, int n_, int k_)
      : m(m_), n(n_), k(k_), mp((m_ + 15) & ~15), kp((k_ + 15) & ~15),
        ng(((n_ + 63) & ~63) >> 2), rs(((n_ + 63) & ~63) + 16) {
    na = mp * ng;
    nb = ng * (kp >> 2);
    g16 = ng >> 4;
    rng = 0xFFFFFFFFu / (uint32_t)ng + 1;
    rg16 = g16 > 1 ? 0xFFFFFFFFu / g16 + 1 : 0u;
  }
  __device__ __forceinline__ void a_item(uint32_t f, uint32_t& i, uint32_t& l0) const {
    i = __umulhi(f, rng);
    l0 = (f - i * ng) * 4;
  }
  __device__ __forceinline__ void b_item(uint32_t f, uint32_t& l0, uint32_t& j0) const {
    const uint32_t r = f >> 6, hh = g16 == 1 ? r : __umulhi(r, rg16), gh = r - hh * g16;
    l0 = (gh * 16 + (f & 15)) * 4;
    j0 = (hh * 4 + ((f >> 4) & 3)) * 4;
  }
};

// Every slot issues its loads (an item outside the matrices reads element
// 0 and is zeroed when staged), so the number of loads in flight is a
// compile-time constant and a wait for one buffer never waits for the
// loads issued after it.
template <int NT, int PA, int PB>
__device__ __forceinline__ void pipe_load(PipeRegs<PA, PB>& r, const PipeShape& S,
                                          const uint32_t* A, const uint32_t* B) {
  const uint32_t tid = opaque(threadIdx.x);
#pragma unroll
  for (int s = 0; s < PA; ++s) {
    const uint32_t f = tid + s * NT;
    uint32_t i, l0;
    S.a_item(f, i, l0);
    const bool ok = f < S.na && i < (uint32_t)S.m && l0 < (uint32_t)S.n;
    r.a[s] = *(const uint4*)(A + (ok ? i * (uint32_t)S.n + l0 : 0u));
  }
#pragma unroll
  for (int s = 0; s < PB; ++s) {
    const uint32_t f = tid + s * NT;
    uint32_t l0, j0;
    S.b_item(f, l0, j0);
    const bool ok = f < S.nb && j0 < (uint32_t)S.k && l0 < (uint32_t)S.n;
    const uint32_t o = ok ? l0 * (uint32_t)S.k + j0 : 0u, dk = ok ? (uint32_t)S.k : 0u;
#pragma unroll
    for (int c = 0; c < 4; ++c) r.b[s][c] = *(const uint4*)(B + (o + c * dk));
  }
}

// Limb planes of the point held in r, written to LDS (items outside the
// matrices as zeros).
template <bool CENTER, int NT, int PA, int PB>
__device__ __forceinline__ void pipe_stage(const PipeRegs<PA, PB>& r, const PipeShape& S,
                                           uint8_t* As, uint8_t* Bs, uint32_t q,
                                           uint32_t half_q) {
  const uint32_t tid = opaque(threadIdx.x);
#pragma unroll
  for (int s = 0; s < PA; ++s) {
    const uint32_t f = tid + s * NT;
    if (f < S.na) {
      uint32_t i, l0;
      S.a_item(f, i, l0);
      const bool ok = i < (uint32_t)S.m && l0 < (uint32_t)S.n;
      uint32_t in[4] = {ok ? limbs_of<CENTER>(r.a[s].x, q, half_q) : 0u,
                        ok ? limbs_of<CENTER>(r.a[s].y, q, half_q) : 0u,
                        ok ? limbs_of<CENTER>(r.a[s].z, q, half_q) : 0u,
                        ok ? limbs_of<CENTER>(r.a[s].w, q, half_q) : 0u};
      uint32_t out[4];
      transpose4x4(in, out);
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) *(uint32_t*)(As + (pl * S.mp + i) * S.rs + l0) = out[pl];
    }
  }
#pragma unroll
  for (int s = 0; s < PB; ++s) {
    const uint32_t f = tid + s * NT;
    if (f < S.nb) {
      uint32_t l0, j0;
      S.b_item(f, l0, j0);
      const bool ok = j0 < (uint32_t)S.k && l0 < (uint32_t)S.n;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {  // column j0 + cc: its rows l0 .. l0 + 3
        uint32_t in[4], out[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t w = cc == 0 ? r.b[s][c].x : cc == 1 ? r.b[s][c].y
                           : cc == 2 ? r.b[s][c].z : r.b[s][c].w;
          in[c] = ok ? limbs_of<CENTER>(w, q, half_q) : 0u;
        }
        transpose4x4(in, out);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
          *(uint32_t*)(Bs + (pl * S.kp + j0 + cc) * S.rs + l0) = out[pl];
      }
    }
  }
}

// Points t0, t0 + ts, ... below t1; the next point loads while the matrix
// cores work on this one.  (A second register buffer, so that the load
// starts before this point's limb planes are written, measured no faster.)
template <bool CENTER, int NT, int PA, int PB>
__device__ __forceinline__ void pointwise_mfma_pipe(const PointwiseLaunch& a, int prime,
                                                    uint32_t t0, uint32_t t1, uint32_t ts,
                                                    uint32_t* smem) {
  const uint32_t q = a.pc[prime].q, half_q = q >> 1;
  const PipeShape S(a.m, a.n, a.k);
  const int np = S.ng * 4;
  uint8_t* As = (uint8_t*)smem;
  uint8_t* Bs = As + 4 * S.mp * S.rs;
  const uint32_t* A0 = a.ahat + a.a_prime_stride * prime;
  const uint32_t* B0 = a.bhat + a.b_prime_stride * prime;
  const size_t mn = (size_t)a.m * a.n, nk = (size_t)a.n * a.k;
  if (t0 >= t1) return;
  PipeRegs<PA, PB> r;
  pipe_load<NT>(r, S, A0 + t0 * mn, B0 + t0 * nk);
  for (uint32_t t = t0; t < t1; t += ts) {
    lds_barrier();  // the previous point's products have read the planes
    pipe_stage<CENTER, NT>(r, S, As, Bs, q, half_q);
    lds_barrier();
    if (t + ts < t1) pipe_load<NT>(r, S, A0 + (t + ts) * mn, B0 + (t + ts) * nk);
    mfma_point(a, t, prime, As, Bs, S.mp, S.kp, np, S.rs);
  }
}

// The pipelined kernel for a shape: 1 (PA = 4, PB = 1), 2 (8, 2).
template <int NT, int PA, int PB>
__device__ __forceinline__ void pointwise_mfma_pipe_any(const PointwiseLaunch& a, int prime,
                                                        uint32_t t0, uint32_t t1, uint32_t ts,
                                                        uint32_t* smem) {
  if (a.pc[prime].q <= 0x7F7F7F7Fu)
    pointwise_mfma_pipe<false, NT, PA, PB>(a, prime, t0, t1, ts, smem);
  else
    pointwise_mfma_pipe<true, NT, PA, PB>(a, prime, t0, t1, ts, smem);
}

}  // namespace pm
