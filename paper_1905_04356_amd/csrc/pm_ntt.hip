// pm_ntt.hip -- single-product transform kernels and their launchers.
//
// The device work of each workgroup lives in pm_ntt_dev.h; this file wraps
// it in one kernel per tile kind and launches one product's transforms.
#include <algorithm>

#include "pm_batch.h"
#include "pm_ntt_dev.h"
#include "pm_profile.h"

namespace pm {

template <typename TIn, bool REDUCE, int V>
__global__ __launch_bounds__(kNT) void ntt_fwd_kernel(NttLaunch a) {
  extern __shared__ uint32_t lds[];
  fwd_lds_tile<TIn, REDUCE, V>(a, blockIdx.y, xcd_block(blockIdx.x, gridDim.x), lds);
}

template <typename TOut, int V>
__global__ __launch_bounds__(kNT) void ntt_inv_kernel(NttLaunch a) {
  extern __shared__ uint32_t lds[];
  inv_lds_tile<TOut, V>(a, blockIdx.y, xcd_block(blockIdx.x, gridDim.x), lds);
}

template <bool DIF, int V, int NT>
__global__ __launch_bounds__(NT, 4) void ntt_block_kernel(NttLaunch a) {
  extern __shared__ uint32_t lds[];
  block_tile<DIF, V, NT>(a, blockIdx.y, xcd_block(blockIdx.x, gridDim.x), blockIdx.z, lds);
}

template <bool DIF, int NT, int PT, int R1, int R2, int R3>
__global__ __launch_bounds__(NT, 4) void ntt_block_regc_kernel(NttLaunch a) {
  extern __shared__ uint32_t lds[];
  block_tile_regc<DIF, NT, PT, R1, R2, R3>(a, blockIdx.y, xcd_block(blockIdx.x, gridDim.x),
                                           blockIdx.z, lds);
}

template <typename TIn, bool REDUCE, int r>
__global__ __launch_bounds__(kColNT) void ntt_col_fwd_kernel(NttLaunch a) {
  col_fwd_tile<TIn, REDUCE, r>(a, blockIdx.y, blockIdx.x * kColNT + threadIdx.x, col_items(a),
                               gridDim.x * kColNT);
}

// The forward transforms of both operands of a product in one launch per
// step (their split transforms share the pass structure and, for the block
// step, the register tile): the first nb_a workgroups (first pass) or
// entry blocks (block step) take operand a, the rest operand b.  One launch
// of both keeps the device fuller than two (the first pass of configuration
// 2's operands, 4096 and 2048 entries, runs at 4.7 and 4.4 TB/s alone).
template <typename TIn, bool REDUCE, int r>
__global__ __launch_bounds__(kColNT) void ntt_col_fwd_pair_kernel(NttLaunch a, NttLaunch b,
                                                                  uint32_t nb_a) {
  if (blockIdx.x < nb_a)
    col_fwd_tile<TIn, REDUCE, r>(a, blockIdx.y, blockIdx.x * kColNT + threadIdx.x, col_items(a),
                                 nb_a * kColNT);
  else
    col_fwd_tile<TIn, REDUCE, r>(b, blockIdx.y, (blockIdx.x - nb_a) * kColNT + threadIdx.x,
                                 col_items(b), (gridDim.x - nb_a) * kColNT);
}

// Unsplit transforms (short lengths): both operands' LDS tiles in one launch.
template <typename TIn, bool REDUCE, int V>
__global__ __launch_bounds__(kNT) void ntt_fwd_pair_kernel(NttLaunch a, NttLaunch b,
                                                           uint32_t nb_a) {
  extern __shared__ uint32_t lds[];
  const uint32_t x = xcd_block(blockIdx.x, gridDim.x);
  if (x < nb_a) fwd_lds_tile<TIn, REDUCE, V>(a, blockIdx.y, x, lds);
  else fwd_lds_tile<TIn, REDUCE, V>(b, blockIdx.y, x - nb_a, lds);
}

template <int V, int NT>
__global__ __launch_bounds__(NT, 4) void ntt_block_pair_kernel(NttLaunch a, NttLaunch b,
                                                              uint32_t nb_a) {
  extern __shared__ uint32_t lds[];
  const uint32_t x = xcd_block(blockIdx.x, gridDim.x);
  if (x < nb_a) block_tile<true, V, NT>(a, blockIdx.y, x, blockIdx.z, lds);
  else block_tile<true, V, NT>(b, blockIdx.y, x - nb_a, blockIdx.z, lds);
}

template <int NT, int PT, int R1, int R2, int R3>
__global__ __launch_bounds__(NT, 4) void ntt_block_regc_pair_kernel(NttLaunch a, NttLaunch b,
                                                                   uint32_t nb_a) {
  extern __shared__ uint32_t lds[];
  const uint32_t x = xcd_block(blockIdx.x, gridDim.x);
  if (x < nb_a) block_tile_regc<true, NT, PT, R1, R2, R3>(a, blockIdx.y, x, blockIdx.z, lds);
  else block_tile_regc<true, NT, PT, R1, R2, R3>(b, blockIdx.y, x - nb_a, blockIdx.z, lds);
}

// (two waves per SIMD: up to 256 VGPRs for the NP x 2^r residues an item holds)
// CRT mode, the first forward pass of all primes from one read of the input
// (col_fwd_items_mp), for one operand or both (nb_a = gridDim.x: one).
template <typename TIn, int r>
__global__ __launch_bounds__(kColNT) void ntt_col_fwd_mp_kernel(NttLaunch a, NttLaunch b,
                                                                uint32_t nb_a, int nprimes) {
  if (blockIdx.x < nb_a)
    col_fwd_tile_mp<TIn, r>(a, nprimes, blockIdx.x * kColNT + threadIdx.x, col_items(a),
                            nb_a * kColNT);
  else
    col_fwd_tile_mp<TIn, r>(b, nprimes, (blockIdx.x - nb_a) * kColNT + threadIdx.x,
                            col_items(b), (gridDim.x - nb_a) * kColNT);
}

template <typename TOut, int r, int NP, bool TR, bool LAZYIN>
__global__ __launch_bounds__(kColNT, 2) void ntt_col_inv_crt_kernel(NttLaunch a, CrtLaunch c) {
  const uint32_t items = (1u << (a.logL - r)) * (uint32_t)a.E;
  col_inv_crt_items<TOut, r, NP, TR, LAZYIN>(a, c, blockIdx.x * kColNT + threadIdx.x, items,
                                             gridDim.x * kColNT);
}

template <typename TOut, int r>
__global__ __launch_bounds__(kColNT) void ntt_col_inv_kernel(NttLaunch a) {
  col_inv_tile<TOut, r>(a, blockIdx.y, blockIdx.x * kColNT + threadIdx.x, col_items(a),
                        gridDim.x * kColNT);
}

// ---- host side ---------------------------------------------------------------

void fill_ntt_launch(NttLaunch* a, int logL, int E, int nin, int io_bytes, bool inverse,
                     bool batched, const Knobs& kn) {
  const PassPlan PP = make_pass_plan(logL, kn.split, kn.maxr);
  a->logL = logL;
  a->npass = PP.npass;
  a->split = PP.split;
  a->blk_log = logL - PP.split;
  for (int i = 0; i < kMaxPasses; ++i) {
    a->stages[i] = i < PP.npass ? PP.stages[i] : 0;
    a->stride_log[i] = i < PP.npass ? PP.stride_log[i] : 0;
    a->tw_off[i] = i < PP.npass ? PP.tw_off[i] : 0;
  }
  a->keep = PP.split ? 1 << PP.split : 1;
  a->lazy = 0;
  a->nin = nin;
  a->out_lo = 0;
  a->E = E;
  // about 2^lds_log residues of LDS per workgroup, at least one entry, no
  // more slots than entries
  const GlobalKnobs G = global_knobs();
  const int tile_log = inverse && kn.blk_tile_log_inv ? kn.blk_tile_log_inv : kn.blk_tile_log;
  const int blk_nt = inverse && kn.blk_nt_inv ? kn.blk_nt_inv : kn.blk_nt;
  int eb = (PP.split ? (batched ? G.batch_tile_log : tile_log) : G.lds_log) - a->blk_log;
  if (eb < 0) eb = 0;
  while (eb > 0 && (1 << (eb - 1)) >= E) --eb;
  // A single product with few entries takes fewer entries per workgroup,
  // down to one, while its launch would have fewer than min_wg workgroups:
  // such transforms are latency-bound (a full-size register tile is kept).
  // Unsplit lengths have their own bound: fewer entries per workgroup there
  // also narrows the vectors of the LDS tile's loads.
  const int min_wg = PP.split ? G.min_wg : G.min_wg_unsplit;
  if (!batched && min_wg > 0) {
    const int nt_log = blk_nt == 512 ? 9 : 8;
    const bool full_reg = PP.split && kn.reg_tile && a->blk_log + eb == nt_log + 5;
    const long zb = PP.split ? 1L << PP.split : 1;
    while (eb > 0 && !full_reg && ((E + (1L << eb) - 1) >> eb) * zb < min_wg) --eb;
  }
  a->eb_log = eb;
  // entries move between HBM and LDS in vectors of V consecutive residues
  int v = 4;
  while (v > 1 && ((E % v) != 0 || (1 << eb) % v != 0)) v >>= 1;
  a->vec = v;
  // column items move at most 16 bytes per row access
  int cv = inverse ? kn.colvec_inv : kn.colvec_fwd;
  if (cv == 3) cv = 2;
  if (PP.split >= 5 && cv > 2) cv = 2;  // 32 residues per entry
  // inputs longer than L/2 take the one-entry full-load column pass
  if (!inverse && 2 * nin > (1 << logL)) cv = 1;
  while (cv > 1 && ((E % cv) != 0 || cv * io_bytes > 16)) cv >>= 1;
  a->col_vec = cv;
  const int B = 1 << a->blk_log;
  a->lds_stride = B + (B >> 5) + 1;
  a->blk_pitch = ((1 << eb) + 3) / 4 * 4 + G.blk_pad;
  // the register tile, for the threads that run the block step: kBatchNT in
  // the batched phase kernels, blk_nt in the single-product kernel
  a->blk_nt = batched ? kBatchNT : blk_nt;
  const int nt_log = a->blk_nt == 512 ? 9 : 8;
  a->reg_kind = kn.reg_tile ? reg_kind_of(*a, nt_log) : 0;
}

static size_t lds_bytes(const NttLaunch& a) {
  return sizeof(uint32_t) * (size_t)a.lds_stride << a.eb_log;
}

template <typename K>
static int launch_lds(K kernel, const NttLaunch& a, int nprimes, int zblocks, hipStream_t s,
                      size_t lds, int nt = kNT) {
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int EB = 1 << a.eb_log;
  dim3 grid((a.E + EB - 1) / EB, nprimes, zblocks);
  return launch(kernel, grid, dim3(nt), lds, s, a);
}

template <typename K>
static int launch_col(K kernel, const NttLaunch& a, int nprimes, hipStream_t s) {
  const uint64_t items = col_items(a);
  uint64_t blocks = (items + kColNT - 1) / kColNT;
  if (blocks > 8192) blocks = 8192;
  return launch(kernel, dim3((unsigned)blocks, nprimes), dim3(kColNT), 0, s, a);
}

static uint32_t col_blocks(const NttLaunch& a) {
  const uint64_t blocks = (col_items(a) + (uint64_t)kColNT - 1) / kColNT;
  return (uint32_t)(blocks > 8192 ? 8192 : blocks);
}

// CRT mode with several primes and inputs within L/2 rows: the first pass of
// every prime from one read of the input (global knob col_fwd_mp).
template <bool REDUCE>
static bool col_mp_ok(const NttLaunch& a, int nprimes) {
  return REDUCE && nprimes > 1 && a.in_prime_stride == 0 && 2 * a.nin <= (1 << a.logL) &&
         global_knobs().col_fwd_mp;
}

// The multi-prime first pass of a (nb = 0) or of a and b.
template <typename TIn>
static int launch_col_mp(const NttLaunch& a, const NttLaunch* b, int nprimes, hipStream_t s) {
  const uint32_t na = col_blocks(a), nb = b ? col_blocks(*b) : 0;
  const NttLaunch& bb = b ? *b : a;
  const dim3 grid(na + nb);
  switch (a.split) {
    case 2: return launch(ntt_col_fwd_mp_kernel<TIn, 2>, grid, dim3(kColNT), 0, s, a, bb, na, nprimes);
    case 3: return launch(ntt_col_fwd_mp_kernel<TIn, 3>, grid, dim3(kColNT), 0, s, a, bb, na, nprimes);
    case 5: return launch(ntt_col_fwd_mp_kernel<TIn, 5>, grid, dim3(kColNT), 0, s, a, bb, na, nprimes);
    default: return launch(ntt_col_fwd_mp_kernel<TIn, 4>, grid, dim3(kColNT), 0, s, a, bb, na, nprimes);
  }
}

template <typename TIn, bool REDUCE>
static int launch_col_fwd_r(const NttLaunch& a, int nprimes, hipStream_t s) {
  if (col_mp_ok<REDUCE>(a, nprimes)) return launch_col_mp<TIn>(a, nullptr, nprimes, s);
  switch (a.split) {
    case 2: return launch_col(ntt_col_fwd_kernel<TIn, REDUCE, 2>, a, nprimes, s);
    case 3: return launch_col(ntt_col_fwd_kernel<TIn, REDUCE, 3>, a, nprimes, s);
    case 5: return launch_col(ntt_col_fwd_kernel<TIn, REDUCE, 5>, a, nprimes, s);
    default: return launch_col(ntt_col_fwd_kernel<TIn, REDUCE, 4>, a, nprimes, s);
  }
}

template <typename TOut>
static int launch_col_inv_r(const NttLaunch& a, int nprimes, hipStream_t s) {
  switch (a.split) {
    case 2: return launch_col(ntt_col_inv_kernel<TOut, 2>, a, nprimes, s);
    case 3: return launch_col(ntt_col_inv_kernel<TOut, 3>, a, nprimes, s);
    case 5: return launch_col(ntt_col_inv_kernel<TOut, 5>, a, nprimes, s);
    default: return launch_col(ntt_col_inv_kernel<TOut, 4>, a, nprimes, s);
  }
}

// The register-resident block step of a launch with reg_kind set.
template <bool DIF, int NT>
static int launch_reg(const NttLaunch& a, int nprimes, int zb, hipStream_t s, size_t lds) {
  switch (a.reg_kind) {
    case 1: return launch_lds(ntt_block_regc_kernel<DIF, NT, 8, 3, 3, 3>, a, nprimes, zb, s, lds, NT);
    case 2: return launch_lds(ntt_block_regc_kernel<DIF, NT, 16, 4, 3, 0>, a, nprimes, zb, s, lds, NT);
    case 3: return launch_lds(ntt_block_regc_kernel<DIF, NT, 16, 4, 4, 0>, a, nprimes, zb, s, lds, NT);
    case 4: return launch_lds(ntt_block_regc_kernel<DIF, NT, 16, 4, 3, 3>, a, nprimes, zb, s, lds, NT);
    case 5: return launch_lds(ntt_block_regc_kernel<DIF, NT, 16, 4, 4, 3>, a, nprimes, zb, s, lds, NT);
    default: return hipErrorInvalidValue;
  }
}

template <bool DIF>
static int launch_block(const NttLaunch& a, int nprimes, hipStream_t s) {
  const int zb = a.keep;
  const size_t lds = block_lds_bytes(a);
  if (a.reg_kind)
    return a.blk_nt == 256 ? launch_reg<DIF, 256>(a, nprimes, zb, s, lds)
                           : launch_reg<DIF, kNT>(a, nprimes, zb, s, lds);
  if (a.blk_nt == 256) {
    if (a.vec == 4) return launch_lds(ntt_block_kernel<DIF, 4, 256>, a, nprimes, zb, s, lds, 256);
    if (a.vec == 2) return launch_lds(ntt_block_kernel<DIF, 2, 256>, a, nprimes, zb, s, lds, 256);
    return launch_lds(ntt_block_kernel<DIF, 1, 256>, a, nprimes, zb, s, lds, 256);
  }
  if (a.vec == 4) return launch_lds(ntt_block_kernel<DIF, 4, kNT>, a, nprimes, zb, s, lds);
  if (a.vec == 2) return launch_lds(ntt_block_kernel<DIF, 2, kNT>, a, nprimes, zb, s, lds);
  return launch_lds(ntt_block_kernel<DIF, 1, kNT>, a, nprimes, zb, s, lds);
}

template <typename TIn, bool REDUCE>
static int launch_fwd_t(const NttLaunch& a, int nprimes, hipStream_t s) {
  if (a.split) {
    int st = launch_col_fwd_r<TIn, REDUCE>(a, nprimes, s);
    if (st != hipSuccess) return st;
    return launch_block<true>(a, nprimes, s);
  }
  // 32-bit inputs move in 16-byte vectors when E allows, 64-bit ones in 16 bytes
  constexpr int VW = sizeof(TIn) == 4 ? 4 : 2;
  if (a.vec >= VW) return launch_lds(ntt_fwd_kernel<TIn, REDUCE, VW>, a, nprimes, 1, s, lds_bytes(a));
  return launch_lds(ntt_fwd_kernel<TIn, REDUCE, 1>, a, nprimes, 1, s, lds_bytes(a));
}

int launch_ntt_fwd(const NttLaunch& a, int elem_bytes, int reduce, int nprimes,
                   hipStream_t s) {
  if (elem_bytes == 8) return launch_fwd_t<uint64_t, true>(a, nprimes, s);
  if (reduce) return launch_fwd_t<uint32_t, true>(a, nprimes, s);
  return launch_fwd_t<uint32_t, false>(a, nprimes, s);
}

// ---- both operands in one launch per step ------------------------------------

bool ntt_fwd_pair_ok(const NttLaunch& a, const NttLaunch& b) {
  if (!a.split && !b.split)  // unsplit: one LDS kernel per operand, same passes
    return a.logL == b.logL && a.npass == b.npass;
  if (!a.split || a.split != b.split || a.logL != b.logL || a.keep != b.keep ||
      a.npass != b.npass || a.reg_kind != b.reg_kind || a.blk_nt != b.blk_nt)
    return false;
  // the register tile fixes the entries per tile; LDS tiles may differ
  if (a.reg_kind && (a.eb_log != b.eb_log || a.blk_pitch != b.blk_pitch)) return false;
  for (int i = 0; i < a.npass; ++i)
    if (a.stages[i] != b.stages[i] || a.stride_log[i] != b.stride_log[i]) return false;
  return true;
}


template <typename TIn, bool REDUCE>
static int launch_col_pair(const NttLaunch& a, const NttLaunch& b, int nprimes, hipStream_t s) {
  if (col_mp_ok<REDUCE>(a, nprimes) && col_mp_ok<REDUCE>(b, nprimes))
    return launch_col_mp<TIn>(a, &b, nprimes, s);
  const uint32_t na = col_blocks(a), nb = col_blocks(b);
  const dim3 grid(na + nb, nprimes);
  switch (a.split) {
    case 2: return launch(ntt_col_fwd_pair_kernel<TIn, REDUCE, 2>, grid, dim3(kColNT), 0, s, a, b, na);
    case 3: return launch(ntt_col_fwd_pair_kernel<TIn, REDUCE, 3>, grid, dim3(kColNT), 0, s, a, b, na);
    case 5: return launch(ntt_col_fwd_pair_kernel<TIn, REDUCE, 5>, grid, dim3(kColNT), 0, s, a, b, na);
    default: return launch(ntt_col_fwd_pair_kernel<TIn, REDUCE, 4>, grid, dim3(kColNT), 0, s, a, b, na);
  }
}

template <int NT, int PT, int R1, int R2, int R3>
static int launch_reg_pair_t(const NttLaunch& a, const NttLaunch& b, int nprimes,
                             hipStream_t s) {
  const size_t lds = block_lds_bytes(a);
  auto kernel = ntt_block_regc_pair_kernel<NT, PT, R1, R2, R3>;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int EB = 1 << a.eb_log;
  const uint32_t na = (a.E + EB - 1) / EB, nb = (b.E + EB - 1) / EB;
  return launch(kernel, dim3(na + nb, nprimes, a.keep), dim3(NT), lds, s, a, b, na);
}

template <int NT>
static int launch_reg_pair(const NttLaunch& a, const NttLaunch& b, int nprimes, hipStream_t s) {
  switch (a.reg_kind) {
    case 1: return launch_reg_pair_t<NT, 8, 3, 3, 3>(a, b, nprimes, s);
    case 2: return launch_reg_pair_t<NT, 16, 4, 3, 0>(a, b, nprimes, s);
    case 3: return launch_reg_pair_t<NT, 16, 4, 4, 0>(a, b, nprimes, s);
    case 4: return launch_reg_pair_t<NT, 16, 4, 3, 3>(a, b, nprimes, s);
    case 5: return launch_reg_pair_t<NT, 16, 4, 4, 3>(a, b, nprimes, s);
    default: return hipErrorInvalidValue;
  }
}

template <int V, int NT>
static int launch_block_pair_v(const NttLaunch& a, const NttLaunch& b, int nprimes,
                               hipStream_t s) {
  const size_t lds = std::max(block_lds_bytes(a), block_lds_bytes(b));
  auto kernel = ntt_block_pair_kernel<V, NT>;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const uint32_t na = (a.E + (1 << a.eb_log) - 1) >> a.eb_log;
  const uint32_t nb = (b.E + (1 << b.eb_log) - 1) >> b.eb_log;
  return launch(kernel, dim3(na + nb, nprimes, a.keep), dim3(NT), lds, s, a, b, na);
}

// LDS-tile block steps of both operands: vectors of the width both allow.
template <int NT>
static int launch_block_pair(const NttLaunch& a, const NttLaunch& b, int nprimes,
                             hipStream_t s) {
  const int v = std::min(a.vec, b.vec);
  if (v == 4) return launch_block_pair_v<4, NT>(a, b, nprimes, s);
  if (v == 2) return launch_block_pair_v<2, NT>(a, b, nprimes, s);
  return launch_block_pair_v<1, NT>(a, b, nprimes, s);
}

template <typename TIn, bool REDUCE, int V>
static int launch_lds_pair_v(const NttLaunch& a, const NttLaunch& b, int nprimes,
                             hipStream_t s) {
  const size_t lds = std::max(lds_bytes(a), lds_bytes(b));
  auto kernel = ntt_fwd_pair_kernel<TIn, REDUCE, V>;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const uint32_t na = (a.E + (1 << a.eb_log) - 1) >> a.eb_log;
  const uint32_t nb = (b.E + (1 << b.eb_log) - 1) >> b.eb_log;
  return launch(kernel, dim3(na + nb, nprimes), dim3(kNT), lds, s, a, b, na);
}

template <typename TIn, bool REDUCE>
static int launch_fwd_pair_t(const NttLaunch& a, const NttLaunch& b, int nprimes,
                             hipStream_t s) {
  if (!a.split) {
    // 32-bit inputs move in 16-byte vectors where both operands allow, 64-bit in 16 bytes
    constexpr int VW = sizeof(TIn) == 4 ? 4 : 2;
    if (a.vec >= VW && b.vec >= VW) return launch_lds_pair_v<TIn, REDUCE, VW>(a, b, nprimes, s);
    return launch_lds_pair_v<TIn, REDUCE, 1>(a, b, nprimes, s);
  }
  int st = launch_col_pair<TIn, REDUCE>(a, b, nprimes, s);
  if (st != hipSuccess) return st;
  if (!a.reg_kind)
    return a.blk_nt == 256 ? launch_block_pair<256>(a, b, nprimes, s)
                           : launch_block_pair<kNT>(a, b, nprimes, s);
  return a.blk_nt == 256 ? launch_reg_pair<256>(a, b, nprimes, s)
                         : launch_reg_pair<kNT>(a, b, nprimes, s);
}

int launch_ntt_fwd_pair(const NttLaunch& a, const NttLaunch& b, int elem_bytes, int reduce,
                        int nprimes, hipStream_t s) {
  if (!ntt_fwd_pair_ok(a, b)) return hipErrorInvalidValue;
  if (elem_bytes == 8) return launch_fwd_pair_t<uint64_t, true>(a, b, nprimes, s);
  if (reduce) return launch_fwd_pair_t<uint32_t, true>(a, b, nprimes, s);
  return launch_fwd_pair_t<uint32_t, false>(a, b, nprimes, s);
}

// Split inverse: the block kernel works in place on the evaluation buffer
// a.in, then the column kernel writes the coefficients.
template <typename TOut>
static int launch_inv_t(const NttLaunch& a, int nprimes, hipStream_t s) {
  if (a.split) {
    NttLaunch b = a;
    b.out = (void*)a.in;
    b.out_prime_stride = a.in_prime_stride;
    int st = launch_block<false>(b, nprimes, s);
    if (st != hipSuccess) return st;
    return launch_col_inv_r<TOut>(a, nprimes, s);
  }
  constexpr int VW = sizeof(TOut) == 4 ? 4 : 2;
  if (a.vec >= VW) return launch_lds(ntt_inv_kernel<TOut, VW>, a, nprimes, 1, s, lds_bytes(a));
  return launch_lds(ntt_inv_kernel<TOut, 1>, a, nprimes, 1, s, lds_bytes(a));
}

int launch_ntt_inv(const NttLaunch& a, int out_elem_bytes, int nprimes, hipStream_t s) {
  if (out_elem_bytes == 8) return launch_inv_t<uint64_t>(a, nprimes, s);
  return launch_inv_t<uint32_t>(a, nprimes, s);
}

// ---- inverse transforms with the Chinese remaindering folded in ---------------

// Five primes' 16 residues per item (a 4-stage pass at full length) exceed
// the register file at two waves per SIMD and spill: measured slower than
// the separate kernels (configuration 4: 0.326 vs 0.319 ms), so not fused.
bool ntt_inv_crt_ok(const NttLaunch& a, int nprimes, int out_elem_bytes) {
  if (a.split != 3 && a.split != 4) return false;
  if (a.split == 4 && nprimes == 5 && a.keep == 16) return false;
  if (out_elem_bytes == 4) return nprimes == 2 || nprimes == 3;
  return nprimes >= 2 && nprimes <= 5;
}

template <typename TOut, int r, int NP, bool LAZYIN>
static int launch_inv_crt_rl(const NttLaunch& a, const CrtLaunch& c, hipStream_t s) {
  const uint64_t items = ((uint64_t)1 << (a.logL - r)) * (uint64_t)a.E;
  uint64_t blocks = (items + kColNT - 1) / kColNT;
  if (blocks > 8192) blocks = 8192;
  const bool tr = a.keep < (1 << r);
  if (tr)
    return launch(ntt_col_inv_crt_kernel<TOut, r, NP, true, LAZYIN>, dim3((unsigned)blocks),
                  dim3(kColNT), 0, s, a, c);
  return launch(ntt_col_inv_crt_kernel<TOut, r, NP, false, LAZYIN>, dim3((unsigned)blocks),
                dim3(kColNT), 0, s, a, c);
}

// the register-tile block step before the pass leaves lazy residues in [0, 2q)
template <typename TOut, int r, int NP>
static int launch_inv_crt_r(const NttLaunch& a, const CrtLaunch& c, hipStream_t s) {
  if (a.lazy && a.reg_kind) return launch_inv_crt_rl<TOut, r, NP, true>(a, c, s);
  return launch_inv_crt_rl<TOut, r, NP, false>(a, c, s);
}

template <typename TOut, int NP>
static int launch_inv_crt_np(const NttLaunch& a, const CrtLaunch& c, hipStream_t s) {
  return a.split == 3 ? launch_inv_crt_r<TOut, 3, NP>(a, c, s)
                      : launch_inv_crt_r<TOut, 4, NP>(a, c, s);
}

int launch_ntt_inv_crt(const NttLaunch& a, const CrtLaunch& c, int out_elem_bytes, int nprimes,
                       hipStream_t s) {
  if (!ntt_inv_crt_ok(a, nprimes, out_elem_bytes)) return hipErrorInvalidValue;
  // the block step in place on the evaluations, as in launch_ntt_inv
  NttLaunch b = a;
  b.out = (void*)a.in;
  b.out_prime_stride = a.in_prime_stride;
  int st = launch_block<false>(b, nprimes, s);
  if (st != hipSuccess) return st;
  if (out_elem_bytes == 4)
    return nprimes == 2 ? launch_inv_crt_np<uint32_t, 2>(a, c, s)
                        : launch_inv_crt_np<uint32_t, 3>(a, c, s);
  switch (nprimes) {
    case 2: return launch_inv_crt_np<uint64_t, 2>(a, c, s);
    case 3: return launch_inv_crt_np<uint64_t, 3>(a, c, s);
    case 4: return launch_inv_crt_np<uint64_t, 4>(a, c, s);
    default: return launch_inv_crt_np<uint64_t, 5>(a, c, s);
  }
}

}  // namespace pm
