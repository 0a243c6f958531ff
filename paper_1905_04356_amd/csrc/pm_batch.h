// pm_batch.h -- descriptors of a batched launch: many products of uneven
// shapes and degrees run phase by phase, each phase one launch whose
// workgroups take tiles from all products.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_kernels.h"

namespace pm {

// Launch descriptors of one product (shared by the single-product path and
// the batch builder).
struct ProductLaunches {
  NttLaunch f[2];       // forward transforms of A and B
  NttLaunch ib;         // inverse, LDS block step of a split transform (in place)
  NttLaunch inv;        // inverse, unsplit LDS kernel or column step
  PointwiseLaunch pw;
  CrtLaunch crt;
  int32_t elem_bytes;   // 4 or 8
  int32_t reduce;       // inputs need reduction mod each prime (CRT mode)
  int32_t pointwise;    // 1 = int8-MFMA kernel, 0 = VALU kernel
  int32_t mode;         // 0 direct, 1 CRT
  int32_t pw_staged;    // VALU kernel stages its operands in LDS
  int32_t nprimes;
  int32_t pad[2];
};

// batched: launch parameters for the batched phase kernels.
int fill_product_launches(const Plan& P, const void* A, const void* B, void* C, uint8_t* ws,
                          ProductLaunches* out, bool batched = false);

// Tile kinds, grouped into phases that must run in order.
enum BatchKind : uint16_t {
  BK_FWD_LDS = 0,    // phase 0: unsplit forward transform, x = entry block
  BK_COL_FWD = 1,    // phase 0: column pass, x = item chunk
  BK_BLOCK_FWD = 2,  // phase 1: split forward LDS block, x = entry block, z = position block
  BK_PW = 3,         // phase 2 (or 6): points [x * z, x * z + z)
  BK_BLOCK_INV = 4,  // phase 3: split inverse LDS block
  BK_INV_LDS = 5,    // phase 4: unsplit inverse transform
  BK_COL_INV = 6,    // phase 4: column pass of a split inverse
  BK_CRT = 7,        // phase 5: outputs [x * kCrtChunk, ...)
};
// Phase 6 holds the pointwise tiles of products that take the pipelined
// kernel with 8 A groups per thread (its own launch: its registers allow one
// workgroup per CU); it runs after phase 2, before phase 3.
constexpr int kBatchPhases = 7;
constexpr int kBatchPhaseOrder[kBatchPhases] = {0, 1, 2, 6, 3, 4, 5};
constexpr int kBatchNT = 512;
constexpr uint32_t kColChunk = 4096;
constexpr uint32_t kCrtChunk = 8192;

// A segment: `count` consecutive tiles of one kind, operand and prime of one
// product; tile i of the segment has x = i % nx, z = i / nx.
struct BatchSeg {
  uint32_t first;   // index of the segment's first tile within its phase
  uint32_t prod;
  uint32_t nx;
  uint16_t kind, op;      // op: operand (transforms); pipelined variant (pointwise)
  uint16_t prime, zpts;  // zpts: points per pointwise tile
};

// Launch one phase: `ntiles` workgroups over `nseg` segments (device arrays).
int launch_batch_phase(int phase, const ProductLaunches* prods, const BatchSeg* segs, int nseg,
                       uint32_t ntiles, size_t lds, hipStream_t s);

}  // namespace pm
