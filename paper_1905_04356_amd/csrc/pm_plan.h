// pm_plan.h -- host-side planning for libpm: moduli, transform lengths,
// tables of roots of unity, workspace layout.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <new>

namespace pm {

constexpr int kMaxPrimes = 8;
constexpr int kMaxLogLen = 15;     // transforms are LDS-resident: L <= 2^15
constexpr int kMaxPasses = 6;

// Twiddle pair for Shoup multiplication: w and floor(w * 2^32 / q).
struct Tw {
  uint32_t w, wp;
};

// Pass structure of a length-2^logL transform: the forward (decimation in
// frequency) transform runs stages in passes of r_0, r_1, ... radix-2
// stages; pass i works on groups of 2^r_i elements at stride S_i, with
// S_0 = L / 2^r_0 and S_{i+1} = S_i / 2^r_{i+1} (the last stride is 1).  The
// inverse (decimation in time) runs the same passes in reverse order.
// split > 0: pass 0 (split stages at stride L / 2^split) runs as a streaming
// column kernel; the later passes act on independent blocks of
// L / 2^split consecutive positions, which an LDS kernel transforms in place.
struct PassPlan {
  int logL;
  int split;
  int npass;
  int stages[kMaxPasses];      // forward order
  int stride_log[kMaxPasses];  // log2 S_i, forward order
  uint32_t tw_off[kMaxPasses]; // offset (in Tw units) of pass i's table
  uint32_t tw_count;           // total Tw entries of one direction
};

// Launch-shape choices for one product.  None of them changes a result:
// every combination computes the same residues.  Defaults come from the
// environment (PM_TUNE_*, read once); the tuning table (pm_tune.cpp) may
// override them per (prime class, log2 L, shape bucket).
struct Knobs {
  int split;         // stages of the streaming column pass (0 none, 2..4)
  int maxr;          // most stages per LDS pass (2..4)
  int blk_nt;        // single-product block step: threads (256 or 512)
  int blk_tile_log;  // single-product block step: log2 residues per tile
  int colvec_fwd;    // most entries per column-pass item (1, 2, 4), forward
  int colvec_inv;    // ... inverse
  int reg_tile;      // register-resident block tile where it fits (1) or LDS (0)
  int pointwise;     // 1: int8-MFMA where the shape fits, 0: VALU
  int pw_small_lds;  // largest limb-plane footprint run with 256 threads (bytes)
  int pw_pipe;       // pipelined MFMA pointwise: -1 where it fits, 0 never, 1/2 force
  int blk_nt_inv;    // inverse block step: threads (0: as blk_nt)
  int blk_tile_log_inv;  // inverse block step: log2 residues per tile (0: as blk_tile_log)
};

// Choices that are not per product.
struct GlobalKnobs {
  int lds_log;           // unsplit transforms: log2 residues of LDS per workgroup
  int split_min_log;     // smallest log2 L that is split
  int blk_pad;           // block step: LDS words of padding per position
  int batch_tile_log;    // batched phase kernels: log2 residues per block tile
  int batch_pw_work;     // batched pointwise tiles: multiply-adds per tile
  int batch_pw_pipe_pts; // batched pipelined pointwise tiles: points per tile
  int batch_direct_max;  // batches of at most this many products launch per product
  int batch_graph;       // repeated batches replay as HIP graphs (1)
  int wrap_min_log;      // wrapped form: least j (2^j points)
  int wrap_top_div;      // ... top t <= 2^j / wrap_top_div
  int wrap_min_work_log; // ... (mn + nk + mk) 2^j >= 2^wrap_min_work_log
  int vdm_max_d;         // CRT-mode u32 products with d <= this go through Vandermonde
  int min_wg;            // single-product split transforms: fewer entries per
                         // workgroup while a launch has fewer workgroups than this (0: off)
  int min_wg_unsplit;    // the same for transforms of lengths below the split
  int trunc34;           // three-quarter transforms: 0 off, 1 on (the wrapped form
                         // keeps tops t <= 2^j / wrap_top_div_tr), 2 on, never wrapped
  int wrap_top_div_tr;   // wrapped form where a three-quarter transform applies and
                         // log2 L <= wrap_tr_max_log: top t <= 2^j / wrap_top_div_tr
  int wrap_tr_max_log;
  int crt_fused;         // CRT mode: last inverse pass and reconstruction in one kernel (1)
  int col_fwd_mp;        // CRT mode: each forward first pass for all primes from one read (1)
  int lazy;              // lazy butterflies in register-tile block steps where q allows (1)
  int batch_single_min_log;  // batched calls: products of at least 2^this transform work
                             // ((mn + nk + mk) points primes) run as single products (0: none)
};

// Prime classes of the tuning table: direct mode with q < 2^30, direct mode
// with q >= 2^30, CRT mode.
enum { kClassDirectLt30 = 0, kClassDirectGe30 = 1, kClassCrt = 2 };

// The knobs of a product (entry: index of the tuning-table entry used, -1
// for the defaults).
Knobs tuned_knobs(int pclass, int logL, int m, int n, int k, int* entry);
// The defaults (no table entry) and the global choices of the current table.
Knobs base_knobs();
GlobalKnobs global_knobs();
// Incremented whenever a tuning table is installed.
uint64_t tune_epoch();

PassPlan make_pass_plan(int logL, int split, int maxr);

// Per-prime constants shared by all kernels.
struct PrimeConst {
  uint32_t q;
  uint32_t linv, linv_p;   // L^{-1} mod q and its Shoup companion
  uint32_t i4, i4p;        // w^(L/4) (w the forward L-th root) and its companion
  uint32_t pad;
  uint64_t mu;             // floor((2^64-1)/q) for Barrett reduction
  const Tw* tw_fwd;        // device: forward tables (PassPlan order)
  const Tw* tw_inv;        // device: inverse tables (same indexing, w^-1)
};

struct Plan {
  int mode;              // 0 direct, 1 CRT
  int logL;
  int r;                 // number of primes
  uint32_t q[kMaxPrimes];
  int pointwise;         // 0 VALU, 1 MFMA
  Knobs kn;              // launch shapes (tuning table or defaults)
  int tune_entry;        // tuning-table entry of kn, -1 for the defaults
  // Three-quarter transforms: a whole product with 2d - 1 <= 3L/4 needs only
  // the evaluations at the roots of (x^(L/2) - 1)(x^(L/4) - w^(L/4)), the
  // first 3L/4 points of the bit-reversed order; the column pass drops the
  // rest and the last inverse pass solves for the coefficients from them.
  int trunc;             // 1: three-quarter transform
  int npts;              // evaluation points: L, or 3L/4
  int keep;              // column-pass rows (and position blocks) kept: 2^split or 3/4 of it
  int m, n, k, d;
  // coefficient counts of A and B, and the window [lo, lo + nout) of the
  // product's coefficients that is computed (full product: d, d, 0, 2d-1)
  int da, db, lo, nout;
  uint64_t p;
  int elem_bytes;
  // workspace layout (bytes, from the workspace base)
  uint64_t off_ahat, off_bhat, off_chat;  // per-prime stride below
  uint64_t prime_stride;                  // bytes between primes' eval sets
  uint64_t off_cq;                        // CRT residues: r x nout x m x k u32
  uint64_t ws_bytes;
};

// Status codes mirror pm_status in pm.h.
int make_plan(uint64_t p, int m, int n, int k, int d, int elem_bytes, Plan* out);

// Plan of coefficients lo .. lo + nout - 1 of A B, deg A < da, deg B < db:
// the transform length L only has to exceed both da + db - 2 - lo (so that
// no coefficient of degree >= L wraps onto the window) and lo + nout - 1.
// The middle product of the paper is the case da = c, db = c + d, lo = c,
// nout = d.
int make_slice_plan(uint64_t p, int m, int n, int k, int da, int db, int lo, int nout,
                    int elem_bytes, Plan* out);

// Plan of A B mod (x^L - 1), L = 2^logL >= d (coefficients 0 .. min(L, 2d-1) - 1).
int make_cyclic_plan(uint64_t p, int m, int n, int k, int d, int logL, int elem_bytes,
                     Plan* out);

// Pointwise kernel for an m x n by n x k product per point: 1 int8-MFMA
// (where `want` asks for it and the shape fits), 0 VALU.
int choose_pointwise(int m, int n, int k, int want);

// Pass structure of a plan's transforms.
inline PassPlan plan_passes(const Plan& P) {
  return make_pass_plan(P.logL, P.kn.split, P.kn.maxr);
}

// Host number theory (the library's own; the test oracle has separate code).
bool is_prime_u64(uint64_t n);
uint64_t powmod_u64(uint64_t b, uint64_t e, uint64_t m);
int v2_u64(uint64_t x);

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// A place where host code of the library is about to allocate: throws
// std::bad_alloc when the test hook pm_debug_fail_alloc has armed it (every
// entry point turns that into PM_ENOMEM), else does nothing.
void alloc_point();

// Run an entry point's body; a host allocation failure becomes PM_ENOMEM and
// no exception leaves the library.
template <typename F>
int guarded(F&& body) {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return -3;  // PM_ENOMEM
  } catch (...) {
    return -1;  // PM_EINVAL
  }
}

}  // namespace pm
