// pm_batch.hip -- phase kernels of a batched launch.
//
// A batch of products (as the divide-and-conquer approximant-basis algorithm
// of Section 3 issues them, many shapes and degrees at each level; Hyun,
// Neiger, Schost, ISSAC 2019, Algorithm PM-Basis) runs in six phases:
// forward first pass, forward LDS blocks, pointwise products, inverse LDS
// blocks, inverse last pass, Chinese remaindering.  Each phase is one launch
// in which workgroup b finds its segment by binary search over the segments'
// first-tile indices and runs that tile with the same device code as the
// single-product kernels.  Segments are ordered by decreasing tile cost, so
// the hardware dispatcher hands the largest tiles out first.
//
// Phases are separate launches because the L2 caches of the 8 XCDs are not
// coherent with each other inside a kernel: a dependency between tiles of
// one launch would need an L2 write-back at every release.  Kernel
// boundaries give that ordering for free, and the phases are replayed as one
// HIP graph when a batch repeats.
#include "pm_batch.h"
#include "pm_crt_dev.h"
#include "pm_ntt_dev.h"
#include "pm_pointwise_dev.h"
#include "pm_profile.h"

namespace pm {

__device__ __forceinline__ int find_segment(const BatchSeg* segs, int nseg, uint32_t b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Column items of 1 or 2 consecutive entries (2 where the descriptor's col_vec
// allows).
template <typename TIn, bool RED, int r>
__device__ __forceinline__ void col_fwd_cv(const NttLaunch& a, int prime, uint32_t i0, uint32_t i1,
                                           bool zhi) {
  if (!zhi) {
    col_fwd_items<TIn, RED, r, 1, false>(a, prime, i0, i1, kBatchNT);
  } else if (a.col_vec >= 2) {
    col_fwd_items<TIn, RED, r, 2>(a, prime, i0, i1, kBatchNT);
  } else {
    col_fwd_items<TIn, RED, r, 1>(a, prime, i0, i1, kBatchNT);
  }
}

template <typename TIn, bool RED>
__device__ __forceinline__ void phase0(const NttLaunch& a, const BatchSeg& g, uint32_t x,
                                       uint32_t* lds) {
  if (g.kind == BK_COL_FWD) {
    const uint32_t items = col_items(a);
    const uint32_t i0 = x * kColChunk;
    const uint32_t i1 = i0 + kColChunk < items ? i0 + kColChunk : items;
    // whole products have nin = d <= L/2; coefficient windows may not
    const bool zhi = 2 * a.nin <= (1 << a.logL);
    switch (a.split) {
      case 2: col_fwd_cv<TIn, RED, 2>(a, g.prime, i0 + threadIdx.x, i1, zhi); break;
      case 3: col_fwd_cv<TIn, RED, 3>(a, g.prime, i0 + threadIdx.x, i1, zhi); break;
      default: col_fwd_cv<TIn, RED, 4>(a, g.prime, i0 + threadIdx.x, i1, zhi); break;
    }
  } else {
    constexpr int VW = sizeof(TIn) == 4 ? 4 : 2;
    if (a.vec >= VW) fwd_lds_tile<TIn, RED, VW>(a, g.prime, x, lds);
    else fwd_lds_tile<TIn, RED, 1>(a, g.prime, x, lds);
  }
}

template <bool DIF>
__device__ __forceinline__ void block_v(const NttLaunch& a, int prime, int x, int z,
                                        uint32_t* lds) {
  if (a.reg_kind) block_tile_reg_kind<DIF, kBatchNT>(a, prime, x, z, lds);
  else if (a.vec == 4) block_tile<DIF, 4, kBatchNT, 2>(a, prime, x, z, lds);
  else if (a.vec == 2) block_tile<DIF, 2, kBatchNT, 2>(a, prime, x, z, lds);
  else block_tile<DIF, 1, kBatchNT, 2>(a, prime, x, z, lds);
}

template <typename TOut, int r>
__device__ __forceinline__ void col_inv_cv(const NttLaunch& a, int prime, uint32_t i0,
                                           uint32_t i1) {
  const bool tr = a.keep < (1 << r);  // three-quarter transform
  if (a.col_vec >= 2) {
    if (tr) col_inv_items<TOut, r, 2, true>(a, prime, i0, i1, kBatchNT);
    else col_inv_items<TOut, r, 2>(a, prime, i0, i1, kBatchNT);
  } else {
    if (tr) col_inv_items<TOut, r, 1, true>(a, prime, i0, i1, kBatchNT);
    else col_inv_items<TOut, r, 1>(a, prime, i0, i1, kBatchNT);
  }
}

template <typename TOut>
__device__ __forceinline__ void phase4(const NttLaunch& a, const BatchSeg& g, uint32_t x,
                                       uint32_t* lds) {
  if (g.kind == BK_COL_INV) {
    const uint32_t items = col_items(a);
    const uint32_t i0 = x * kColChunk;
    const uint32_t i1 = i0 + kColChunk < items ? i0 + kColChunk : items;
    switch (a.split) {
      case 2: col_inv_cv<TOut, 2>(a, g.prime, i0 + threadIdx.x, i1); break;
      case 3: col_inv_cv<TOut, 3>(a, g.prime, i0 + threadIdx.x, i1); break;
      default: col_inv_cv<TOut, 4>(a, g.prime, i0 + threadIdx.x, i1); break;
    }
  } else {
    constexpr int VW = sizeof(TOut) == 4 ? 4 : 2;
    if (a.vec >= VW) inv_lds_tile<TOut, VW>(a, g.prime, x, lds);
    else inv_lds_tile<TOut, 1>(a, g.prime, x, lds);
  }
}

// The block phases (1, 3) are held to 4 waves per SIMD so that two
// 512-thread workgroups share a CU; the 256-thread pointwise phase to 5,
// as the single-product pointwise kernel runs.  The descriptors are never
// written while a phase runs: __restrict__ lets their fields load into
// scalar registers instead of taking vector registers in every lane.
template <int PHASE, int NT>
__global__ __launch_bounds__(NT, (PHASE == 1 || PHASE == 3) ? 4 : (PHASE == 2 && NT == 256) ? 5 : 1)
void batch_kernel(const ProductLaunches* __restrict__ prods, const BatchSeg* __restrict__ segs,
                  int nseg) {
  extern __shared__ uint32_t lds[];
  const uint32_t b = blockIdx.x;
  const BatchSeg g = segs[find_segment(segs, nseg, b)];
  const ProductLaunches& P = prods[g.prod];
  const uint32_t i = b - g.first;
  const uint32_t x = i % g.nx, z = i / g.nx;
  if (PHASE == 0) {
    const NttLaunch& a = P.f[g.op];
    if (P.elem_bytes == 8) phase0<uint64_t, true>(a, g, x, lds);
    else if (P.reduce) phase0<uint32_t, true>(a, g, x, lds);
    else phase0<uint32_t, false>(a, g, x, lds);
  } else if (PHASE == 1) {
    block_v<true>(P.f[g.op], g.prime, x, z, lds);
  } else if (PHASE == 2 || PHASE == 6) {
    const uint32_t t0 = x * g.zpts;
    uint32_t t1 = t0 + g.zpts;
    if (t1 > (uint32_t)P.pw.L) t1 = P.pw.L;
    if (PHASE == 6) {
      pointwise_mfma_pipe_any<NT, 8, 2>(P.pw, g.prime, t0, t1, 1, lds);
      return;
    }
    if (NT == kBatchNT && g.op == 1) {
      pointwise_mfma_pipe_any<NT, 4, 1>(P.pw, g.prime, t0, t1, 1, lds);
      return;
    }
    for (uint32_t t = t0; t < t1; ++t) {
      if (P.pointwise == 1) pointwise_mfma_tile(P.pw, t, g.prime, lds);
      else if (P.pw_staged) pointwise_valu_tile<true>(P.pw, t, g.prime, lds);
      else pointwise_valu_tile<false>(P.pw, t, g.prime, lds);
      __syncthreads();  // LDS is reused by the next point
    }
  } else if (PHASE == 3) {
    block_v<false>(P.ib, g.prime, x, z, lds);
  } else if (PHASE == 4) {
    if (P.mode == 1 || P.elem_bytes == 4) phase4<uint32_t>(P.inv, g, x, lds);
    else phase4<uint64_t>(P.inv, g, x, lds);
  } else if (PHASE == 5) {
    const uint64_t i0 = (uint64_t)x * kCrtChunk;
    if (P.elem_bytes == 8)
      crt_range<uint64_t>(P.crt, i0 + threadIdx.x, i0 + kCrtChunk, kBatchNT);
    else
      crt_range<uint32_t>(P.crt, i0 + threadIdx.x, i0 + kCrtChunk, kBatchNT);
  }
}

template <int PHASE, int NT>
static int launch_phase_t(const ProductLaunches* prods, const BatchSeg* segs, int nseg,
                          uint32_t ntiles, size_t lds, hipStream_t s) {
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  // Raise the dynamic-LDS limit once, to the whole 160 KiB, on the first
  // launch (which is never inside a graph capture: batches are captured on
  // their second occurrence).
  static const hipError_t attr = hipFuncSetAttribute(
      (const void*)batch_kernel<PHASE, NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
      160 * 1024);
  if (attr != hipSuccess) return attr;
  return launch((batch_kernel<PHASE, NT>), dim3(ntiles), dim3(NT), lds, s, prods, segs,
                     nseg);
}

int launch_batch_phase(int phase, const ProductLaunches* prods, const BatchSeg* segs, int nseg,
                       uint32_t ntiles, size_t lds, hipStream_t s) {
  // The transform tiles are written for kBatchNT threads; pointwise tiles
  // with small limb planes run with 256 threads so more of them share a CU
  // (the single-product launch's rule).
  switch (phase) {
    case 0: return launch_phase_t<0, kBatchNT>(prods, segs, nseg, ntiles, lds, s);
    case 1: return launch_phase_t<1, kBatchNT>(prods, segs, nseg, ntiles, lds, s);
    case 2:
      if (lds <= (size_t)base_knobs().pw_small_lds)
        return launch_phase_t<2, 256>(prods, segs, nseg, ntiles, lds, s);
      return launch_phase_t<2, kBatchNT>(prods, segs, nseg, ntiles, lds, s);
    case 3: return launch_phase_t<3, kBatchNT>(prods, segs, nseg, ntiles, lds, s);
    case 4: return launch_phase_t<4, kBatchNT>(prods, segs, nseg, ntiles, lds, s);
    case 6: return launch_phase_t<6, kBatchNT>(prods, segs, nseg, ntiles, lds, s);
    default: return launch_phase_t<5, kBatchNT>(prods, segs, nseg, ntiles, lds, s);
  }
}

}  // namespace pm
