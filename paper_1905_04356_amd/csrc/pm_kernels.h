// pm_kernels.h -- launch descriptors shared by the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_plan.h"

namespace pm {

// Number-theoretic transforms of E = R*S polynomials (entries) at once.
// Forward: input coefficient-major X[c][e] (c < nin, zero beyond) of TIn,
// reduced mod each prime; output point-major Xhat[t][e] (u32), t < L, in the
// bit-reversed order the in-place decimation-in-frequency passes produce.
// Inverse: input point-major Chat[t][e]; output coefficient-major
// C[c][e] for c < nin (the L^{-1} factor is applied by the pointwise kernel).
// With split > 0 the first forward pass (last inverse pass) is a separate
// streaming kernel and the LDS kernel transforms blocks of 2^blk_log
// positions in place in the point-major buffer.
struct NttLaunch {
  int logL;
  int npass;
  int split;                 // stages of the streaming pass (0: none)
  int blk_log;               // log2 positions per LDS block
  int stages[kMaxPasses];
  int stride_log[kMaxPasses];
  uint32_t tw_off[kMaxPasses];
  int nin;                   // forward: coefficients read; inverse: written
  int out_lo;                // inverse: first coefficient written (to row 0)
  int E;                     // entries per point
  int eb_log;                // log2(entries per workgroup) in the LDS kernel
  int vec;                   // residues per global load/store (1, 2, 4)
  int col_vec;               // column pass: consecutive entries per item (1, 2, 4)
  int blk_pitch;             // block step: LDS words per position (>= 2^eb_log, 4 | pitch)
  int reg_kind;              // block step: 0 LDS-resident tile; 1..5 register-resident
                             // tile with block passes {3,3,3}, {4,3}, {4,4}, {4,3,3},
                             // {4,4,3} (set for the thread count that runs the step)
  int lds_stride;            // 32-bit words between entries in LDS
  int blk_nt;                // single-product block step: threads (256 or 512)
  int lazy;                  // register-tile block steps keep residues in [0, 2q) (moduli
                             // with 2q - 1 <= 0x7F7F7F7F): their outputs feed the pointwise
                             // kernels, or the inverse's last pass, which reduces them
  int keep;                  // split transforms: position blocks transformed, 2^split,
                             // or 3 2^split / 4 for a three-quarter transform (the
                             // column pass then writes, and its inverse reads,
                             // only the rows of those blocks)
  uint64_t in_prime_stride;  // elements between primes' input buffers
  uint64_t out_prime_stride; // elements between primes' output buffers
  const void* in;
  void* out;
  PrimeConst pc[kMaxPrimes];
};

// Pointwise products: for every point t and prime, Chat_t = L^{-1} Ahat_t Bhat_t
// (m x n times n x k), all point-major u32, at the first L points (all of
// them, or 3/4 of them for a three-quarter transform).
struct PointwiseLaunch {
  int m, n, k, L;
  int small_lds;             // limb planes up to this many bytes: 256 threads
  int pipe;                  // pipelined variant: -1 where it fits, 0 never, 1/2 force
  uint64_t prime_stride;     // elements between primes' evaluations of C
  uint64_t a_prime_stride;   // ... of A
  uint64_t b_prime_stride;   // ... of B
  const uint32_t* ahat;
  const uint32_t* bhat;
  uint32_t* chat;
  PrimeConst pc[kMaxPrimes];
  uint32_t cs[kMaxPrimes][8];  // MFMA variant: 256^s L^{-1} 2^32 mod q, s < 7
  uint64_t bias[kMaxPrimes];   // MFMA variant: q * 7 n 2^16, above every |sum|
  uint32_t qninv[kMaxPrimes];  // MFMA variant: -q^{-1} mod 2^32
};

// Chinese remaindering of r residue arrays (u32, `count` each, stride
// `prime_stride` elements) into residues mod p.
struct CrtLaunch {
  int r;
  uint64_t count;
  uint64_t prime_stride;
  const uint32_t* cq;
  void* out;
  uint64_t p;
  double pinv;
  uint32_t q[kMaxPrimes];
  uint32_t mu32[kMaxPrimes];               // floor(2^32 / q_i)
  uint64_t mu_p;                           // floor((2^64-1) / p) (p < 2^32)
  uint32_t inv[kMaxPrimes][kMaxPrimes];    // q_j^{-1} mod q_i (j < i)
  uint32_t inv_p[kMaxPrimes][kMaxPrimes];  // Shoup companions
  uint64_t radix_mod_p[kMaxPrimes];        // prod_{j<i} q_j mod p
};

// Host launchers (return hipError_t as int).
int launch_ntt_fwd(const NttLaunch& a, int elem_bytes, int reduce, int nprimes,
                   hipStream_t s);
int launch_ntt_inv(const NttLaunch& a, int out_elem_bytes, int nprimes, hipStream_t s);
// CRT mode: the inverse transforms of all primes and the Chinese remaindering,
// the last inverse pass and the reconstruction in one kernel (no residue
// arrays in HBM), where supported (ntt_inv_crt_ok: split transforms whose
// first pass has 3 or 4 stages, 2-3 primes for 32-bit outputs, 2-5 for 64-bit,
// not 5 primes with a full 4-stage pass).
bool ntt_inv_crt_ok(const NttLaunch& a, int nprimes, int out_elem_bytes);
int launch_ntt_inv_crt(const NttLaunch& a, const CrtLaunch& c, int out_elem_bytes, int nprimes,
                       hipStream_t s);
// Both operands' forward transforms in one launch per step, where their split
// transforms share the pass structure and register tile (ntt_fwd_pair_ok).
bool ntt_fwd_pair_ok(const NttLaunch& a, const NttLaunch& b);
int launch_ntt_fwd_pair(const NttLaunch& a, const NttLaunch& b, int elem_bytes, int reduce,
                        int nprimes, hipStream_t s);
int launch_pointwise(const PointwiseLaunch& a, int nprimes, hipStream_t s);
// C[i] -= C[off + i] mod p for i < count (elements of elem_bytes bytes).
int launch_unwrap(void* C, uint64_t count, uint64_t off, uint64_t p, int elem_bytes,
                  hipStream_t s);
// Y[i] = (p - X[i]) mod p for i < count (elements of elem_bytes bytes).
int launch_probe_mulhi(uint32_t* out, uint32_t blocks, uint32_t iters, uint32_t m,
                       hipStream_t s);
int launch_neg_mod(uint64_t p, const void* X, void* Y, uint64_t count, int elem_bytes,
                   hipStream_t s);
int launch_pointwise_mfma(const PointwiseLaunch& a, int nprimes, hipStream_t s);
size_t pointwise_mfma_lds(int m, int n, int k);
// Largest pointwise LDS footprint launched with 256 threads (larger: 512).
// Pipelined variant for a shape run with 512 threads: 1 (four register
// slots), 2 (eight) or 0 (none); `knob` -1 where one fits, 0 never, 1 or 2
// that variant where it suffices.
int pointwise_pipe_variant(int m, int n, int k, int knob);
int launch_crt(const CrtLaunch& a, int out_elem_bytes, hipStream_t s);
int launch_check_residues(uint64_t p, const void* x, uint64_t count, int elem_bytes,
                          unsigned long long* counter, hipStream_t s);

// Fill the launch descriptor of a transform for (logL, E, nin).
// io_bytes: bytes per element of the coefficient-major side (the input of a
// forward transform, the output of an inverse one).
// batched: parameters for the batched phase kernels (512-thread block tiles).
// kn: the product's launch shapes (pass structure, tiles, item widths).
void fill_ntt_launch(NttLaunch* a, int logL, int E, int nin, int io_bytes, bool inverse,
                     bool batched, const Knobs& kn);

// LDS bytes of one block-step tile (2^blk_log positions, position-major).
__host__ __device__ inline size_t block_lds_bytes(const NttLaunch& a) {
  return (4ull * (size_t)a.blk_pitch) << a.blk_log;
}

// Work items of the column pass: one per (j < L / 2^split, group of col_vec
// consecutive entries).
__host__ __device__ inline uint32_t col_items(const NttLaunch& a) {
  return (1u << (a.logL - a.split)) * (uint32_t)(a.E / a.col_vec);
}

}  // namespace pm
