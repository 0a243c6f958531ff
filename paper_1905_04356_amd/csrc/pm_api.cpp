// pm_api.cpp -- the C ABI (include/pm.h): argument checks, planning, and the
// launch sequence of one product.
//
// A product runs as (Hyun, Neiger, Schost, ISSAC 2019, Section 2,
// "Polynomial matrix multiplication", evaluation/interpolation):
//   forward transforms of A and B  ->  pointwise matrix products  ->
//   inverse transform of C  [-> Chinese remaindering, for moduli that are
//   not FFT primes].
// All primes of a CRT plan go through each phase in the same launch
// (grid dimension y = prime).
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/pm.h"
#include "pm_batch.h"
#include "pm_kernels.h"
#include "pm_noalloc.h"
#include "pm_plan.h"
#include "pm_profile.h"
#include "pm_tables.h"
#include "pm_vdm.h"

using namespace pm;

static int vdm_check(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d);
static uint64_t vdm_ws_bytes(int m, int n, int k, int d);

// Whether pm_mul_vdm_u32 takes this product (p prime below 2^31, odd,
// 2d - 1 <= min(p, 4095), n < 4096).
static bool vdm_eligible(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d) {
  return p > 2 && vdm_check(p, m, n, k, d) == PM_OK;
}

namespace {
int wrap_log_of(const Plan& P);
int vdm_max_d();
}

static void fill_plan_info(const Plan& P, pm_plan_info* out) {
  memset(out, 0, sizeof *out);
  out->wrap_log2_len = wrap_log_of(P);
  out->mode = P.mode;
  out->log2_len = P.logL;
  out->num_primes = P.r;
  out->pointwise = P.pointwise;
  for (int i = 0; i < P.r; ++i) out->primes[i] = P.q[i];
  out->workspace_bytes = P.ws_bytes;
  out->tune_entry = P.tune_entry;
  out->num_points = P.npts;
}

extern "C" {

const char* pm_status_str(int status) {
  switch (status) {
    case PM_OK: return "PM_OK";
    case PM_EINVAL: return "PM_EINVAL: invalid argument";
    case PM_ERANGE: return "PM_ERANGE: modulus or size out of range";
    case PM_ENOMEM: return "PM_ENOMEM: host allocation failed";
    case PM_EWORKSPACE: return "PM_EWORKSPACE: workspace missing, misaligned or too small";
    case PM_EDEVICE: return "PM_EDEVICE: HIP error";
    case PM_EUNSUPPORTED: return "PM_EUNSUPPORTED: length or bound not supported";
    case PM_EBUSY: return "PM_EBUSY: busy";
    case PM_ETABLES: return "PM_ETABLES: no table region attached, or the regions are full";
    case PM_ESCRATCH:
      return "PM_ESCRATCH: the product needs more than the static scratch of pm_mul_noalloc";
    default: return "unknown pm_status";
  }
}

int pm_abi_version(void) { return PM_ABI_VERSION; }

pm_status pm_plan(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d, int32_t elem_bytes,
                  pm_plan_info* out) {
  return (pm_status)guarded([&] {
    if (!out) return (int)PM_EINVAL;
    Plan P;
    int st = make_plan(p, m, n, k, d, elem_bytes, &P);
    if (st != PM_OK) return st;
    fill_plan_info(P, out);
    if (P.mode == 1 && elem_bytes == 4 && d <= vdm_max_d() && vdm_eligible(p, m, n, k, d))
      out->mode = 2;  // pm_mul_u32 takes the Vandermonde route
    return (int)PM_OK;
  });
}

pm_status pm_workspace_bytes(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                             int32_t elem_bytes, uint64_t* out) {
  return (pm_status)guarded([&] {
    if (!out) return (int)PM_EINVAL;
    Plan P;
    int st = make_plan(p, m, n, k, d, elem_bytes, &P);
    if (st != PM_OK) return st;
    *out = P.ws_bytes;
    return (int)PM_OK;
  });
}

}  // extern "C"

namespace {

bool overlap(const void* a, uint64_t na, const void* b, uint64_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// Checks shared by the single and batched entry points; nothing is enqueued.
int check_operands(const Plan& P, const void* A, const void* B, void* C) {
  if (!A || !B || !C) return PM_EINVAL;
  if (((uintptr_t)A | (uintptr_t)B | (uintptr_t)C) & 15) return PM_EINVAL;
  const uint64_t eb = (uint64_t)P.elem_bytes;
  const uint64_t na = eb * P.da * P.m * P.n, nb = eb * P.db * P.n * P.k;
  const uint64_t nc = eb * (uint64_t)P.nout * P.m * P.k;
  if (overlap(C, nc, A, na) || overlap(C, nc, B, nb)) return PM_EINVAL;
  return PM_OK;
}

int check_workspace(const void* ws, uint64_t ws_bytes, uint64_t need, const void* A,
                    uint64_t na, const void* B, uint64_t nb, const void* C, uint64_t nc) {
  if (!ws || ((uintptr_t)ws & 255)) return PM_EWORKSPACE;
  if (ws_bytes < need) return PM_EWORKSPACE;
  if (overlap(ws, need, A, na) || overlap(ws, need, B, nb) || overlap(ws, need, C, nc))
    return PM_EINVAL;
  return PM_OK;
}

void fill_crt(const Plan& P, CrtLaunch* c) {
  memset(c, 0, sizeof *c);
  c->r = P.r;
  c->p = P.p;
  c->pinv = 1.0 / (double)P.p;
  c->mu_p = ~0ull / P.p;
  for (int i = 0; i < P.r; ++i) {
    const uint32_t qi = P.q[i];
    c->q[i] = qi;
    c->mu32[i] = (uint32_t)((1ull << 32) / qi);
    for (int j = 0; j < i; ++j) {
      const uint32_t inv = (uint32_t)powmod_u64(P.q[j] % qi, qi - 2, qi);
      c->inv[i][j] = inv;
      c->inv_p[i][j] = (uint32_t)(((uint64_t)inv << 32) / qi);
    }
    uint64_t rad = 1 % P.p;
    for (int j = 0; j < i; ++j) rad = (uint64_t)((unsigned __int128)rad * P.q[j] % P.p);
    c->radix_mod_p[i] = rad;
  }
}

}  // namespace

namespace pm {

// Lazy butterflies in the register-tile block steps (global knob lazy): every
// prime with 2q - 1 <= 0x7F7F7F7F, so that 4q < 2^32 and the pointwise
// kernels' digit split (exact up to 0x7F7F7F7F) takes values below 2q.
bool lazy_ok(const Plan& P) {
  if (!global_knobs().lazy) return false;
  for (int i = 0; i < P.r; ++i)
    if (2ull * P.q[i] - 1 > 0x7F7F7F7Full) return false;
  return true;
}

// All launch descriptors of one product; A, B, C device pointers, ws the
// product's workspace (laid out by make_plan).
int fill_product_launches(const Plan& P, const void* A, const void* B, void* C, uint8_t* ws,
                          ProductLaunches* L, bool batched) {
  memset(L, 0, sizeof *L);
  PrimeConst pc[kMaxPrimes];
  for (int i = 0; i < P.r; ++i) {
    int st = prime_const(TwKey{P.q[i], P.logL, P.kn.split, P.kn.maxr}, &pc[i]);
    if (st != PM_OK) return st;
  }
  const int m = P.m, n = P.n, k = P.k;
  const uint64_t pstride = P.prime_stride / 4;  // in u32 elements
  uint32_t* ahat = (uint32_t*)(ws + P.off_ahat);
  uint32_t* bhat = (uint32_t*)(ws + P.off_bhat);
  uint32_t* chat = (uint32_t*)(ws + P.off_chat);
  L->elem_bytes = P.elem_bytes;
  L->reduce = P.mode == 1;  // in direct mode the inputs are already residues mod q = p
  L->pointwise = P.pointwise;
  L->mode = P.mode;
  L->nprimes = P.r;
  L->pw_staged = 4ull * ((uint64_t)m * n + (uint64_t)n * k) <= 128 * 1024;

  NttLaunch& fa = L->f[0];
  fill_ntt_launch(&fa, P.logL, m * n, P.da, P.elem_bytes, false, batched, P.kn);
  for (int i = 0; i < P.r; ++i) fa.pc[i] = pc[i];
  fa.in = A;
  fa.out = ahat;
  fa.in_prime_stride = 0;
  fa.out_prime_stride = pstride;

  NttLaunch& fb = L->f[1];
  fb = fa;
  fill_ntt_launch(&fb, P.logL, n * k, P.db, P.elem_bytes, false, batched, P.kn);
  fb.in = B;
  fb.out = bhat;
  fa.keep = fb.keep = P.keep;
  fa.lazy = fb.lazy = lazy_ok(P);

  PointwiseLaunch& pw = L->pw;
  pw.m = m; pw.n = n; pw.k = k; pw.L = P.npts;
  pw.small_lds = P.kn.pw_small_lds;
  pw.pipe = P.kn.pw_pipe;
  pw.prime_stride = pstride;
  pw.a_prime_stride = pstride;
  pw.b_prime_stride = pstride;
  pw.ahat = ahat; pw.bhat = bhat; pw.chat = chat;
  for (int i = 0; i < P.r; ++i) {
    pw.pc[i] = pc[i];
    // weights of the limb accumulators in Montgomery form:
    // 256^s L^{-1} 2^32 mod q
    uint64_t w = ((uint64_t)pc[i].linv << 32) % P.q[i];
    for (int t = 0; t < 7; ++t) {
      pw.cs[i][t] = (uint32_t)w;
      w = (w << 8) % P.q[i];
    }
    // |sum_s c_s acc_s| < 7 q max|acc_s| <= 7 q n 2^16 (|acc_s| <= 4 n 2^14)
    pw.bias[i] = (uint64_t)P.q[i] * 7ull * (uint64_t)n * 65536ull;
    uint32_t inv = 1;  // q^{-1} mod 2^32 by Newton's iteration (q odd)
    for (int it = 0; it < 5; ++it) inv *= 2u - P.q[i] * inv;
    pw.qninv[i] = 0u - inv;
  }

  NttLaunch& ic = L->inv;
  ic = fa;
  fill_ntt_launch(&ic, P.logL, m * k, P.nout, P.mode == 1 ? 4 : P.elem_bytes, true,
                  batched, P.kn);
  ic.keep = P.keep;
  ic.lazy = lazy_ok(P);
  ic.out_lo = P.lo;
  ic.in = chat;
  ic.in_prime_stride = pstride;
  const uint64_t nout = (uint64_t)P.nout * m * k;
  if (P.mode == 0) {
    ic.out = C;
    ic.out_prime_stride = 0;
  } else {
    ic.out = ws + P.off_cq;
    ic.out_prime_stride = nout;
    CrtLaunch& cr = L->crt;
    fill_crt(P, &cr);
    cr.count = nout;
    cr.prime_stride = nout;
    cr.cq = (const uint32_t*)(ws + P.off_cq);
    cr.out = C;
  }
  // LDS block step of a split inverse: in place on the evaluations of C
  L->ib = ic;
  L->ib.out = chat;
  L->ib.out_prime_stride = pstride;
  return PM_OK;
}

// Twiddle tables of every (prime, length) pair of the plans, on stream s.
int prepare_plans(const Plan* plans, size_t n, hipStream_t s) {
  std::vector<TwKey> keys;
  for (size_t i = 0; i < n; ++i)
    for (int j = 0; j < plans[i].r; ++j)
      keys.push_back(TwKey{plans[i].q[j], plans[i].logL, plans[i].kn.split, plans[i].kn.maxr});
  return prepare_twiddles(keys.data(), (int)keys.size(), s);
}

}  // namespace pm

namespace {

// Enqueue one product from its launch descriptors, one launch (or two for
// split transforms) per phase; skip_fwd[op]: that operand's evaluations are
// given (already pointed to by L.pw).
int launch_product(const Plan& P, const ProductLaunches& L, const bool skip_fwd[2],
                   hipStream_t s) {
  int st;
  if (!skip_fwd[0] && !skip_fwd[1] && ntt_fwd_pair_ok(L.f[0], L.f[1])) {
    KernelTimer kt(K_NTT_FWD, s);
    if (launch_ntt_fwd_pair(L.f[0], L.f[1], P.elem_bytes, L.reduce, P.r, s) != hipSuccess)
      return PM_EDEVICE;
  } else {
    for (int op = 0; op < 2; ++op) {
      if (skip_fwd[op]) continue;
      KernelTimer kt(K_NTT_FWD, s);
      if (launch_ntt_fwd(L.f[op], P.elem_bytes, L.reduce, P.r, s) != hipSuccess)
        return PM_EDEVICE;
    }
  }
  {
    KernelTimer kt(K_POINTWISE, s);
    st = P.pointwise == 1 ? launch_pointwise_mfma(L.pw, P.r, s) : launch_pointwise(L.pw, P.r, s);
    if (st != hipSuccess) return PM_EDEVICE;
  }
  if (P.mode == 1 && global_knobs().crt_fused && ntt_inv_crt_ok(L.inv, P.r, P.elem_bytes)) {
    KernelTimer kt(K_NTT_INV, s);
    if (launch_ntt_inv_crt(L.inv, L.crt, P.elem_bytes, P.r, s) != hipSuccess)
      return PM_EDEVICE;
    return PM_OK;
  }
  {
    KernelTimer kt(K_NTT_INV, s);
    if (launch_ntt_inv(L.inv, P.mode == 0 ? P.elem_bytes : 4, P.r, s) != hipSuccess)
      return PM_EDEVICE;
  }
  if (P.mode == 1) {
    KernelTimer kt(K_CRT, s);
    if (launch_crt(L.crt, P.elem_bytes, s) != hipSuccess) return PM_EDEVICE;
  }
  return PM_OK;
}

int run_product(const Plan& P, const void* A, const void* B, void* C, uint8_t* ws,
                hipStream_t s, bool prepared = false) {
  int st = prepared ? PM_OK : prepare_plans(&P, 1, s);
  if (st != PM_OK) return st;
  ProductLaunches L;
  st = fill_product_launches(P, A, B, C, ws, &L);
  if (st != PM_OK) return st;
  const bool none[2] = {false, false};
  return launch_product(P, L, none, s);
}

// Largest d for which products mod a prime without the needed roots of unity
// go through Vandermonde evaluation on the matrix cores instead of CRT
// (global knob vdm_max_d, default 64: measured faster up to there).
int vdm_max_d() { return global_knobs().vdm_max_d; }

// Products with 2^j < 2d - 1 <= 2^j + 2^(j-1): A B mod (x^(2^j) - 1) on a
// transform of 2^j points, the t = 2d - 1 - 2^j coefficients at and above
// 2^j, which involve only A[h..] and B[h..] (h = 2^j - d + 1), as the window
// t-1 .. 2t-2 of that short product, and the wrapped rows corrected: at most
// 1.5 2^j points instead of 2^(j+1).  The short product and the correction
// cost launches of their own, so this pays only for large products with a
// small top: t <= 2^j / 4 and (mn + nk + mk) 2^j >= 2^25 (measured: 128x128x64
// at t = 103..175 0.60-0.84 of the plain time, 64x64x32 at 2^12 + 103 0.74 and
// 2^12 + 903 0.94; at 2^11 + 151, where (mn + nk + mk) 2^j = 2^24, 1.03; small
// shapes and tops near 2^(j-1) 1.0-2.3).  The bounds are global knobs
// (wrap_min_log, default 10, the least j; wrap_top_div, 4; wrap_min_work_log,
// 25).  Where the product also fits a three-quarter transform (3L/4 points,
// one product, no correction), that is faster from a top of about 2^j / 8
// for L <= 2^13 (L = 2^11..2^13, wrapped time over three-quarter time: at
// t = 0.09 2^j 0.89-0.94 for 128x128x64, 1.01-1.05 for 64x64x{32,64}; at
// 0.16 2^j 1.04-1.09 and 1.15-1.21); for L >= 2^14 the two halves of the wrapped form run on
// transforms of half the length, whose cost per point is lower, and it stays
// ahead over the whole band (0.92-0.99 of the three-quarter time at
// t = 0.24 2^j for L = 2^14, 0.75 for 2^15).  Hence the top bound
// 2^j / wrap_top_div_tr (8) for log2 L <= wrap_tr_max_log (13).
// run_wrapped returns 1 when the product was launched this way, 0 when it
// does not apply, or a pm_status.

// j when a whole product of plan P takes the wrapped form on 2^j points
// (with P's own workspace), else 0; the cyclic and top plans through pc, pt.
int wrap_log_plans(const Plan& P, Plan* pc, Plan* pt) {
  const GlobalKnobs G = global_knobs();
  const int j = P.logL - 1;
  if (P.da != P.db || P.lo != 0 || j < G.wrap_min_log) return 0;
  if (P.trunc && G.trunc34 == 2) return 0;  // the three-quarter transform instead
  const int d = P.d, Lp = 1 << j, t = 2 * d - 1 - Lp;
  const uint64_t entries = (uint64_t)P.m * P.n + (uint64_t)P.n * P.k + (uint64_t)P.m * P.k;
  const int div =
      P.trunc && P.logL <= G.wrap_tr_max_log ? G.wrap_top_div_tr : G.wrap_top_div;
  if (t < 1 || t > Lp / div || d > Lp ||
      (entries << j) < (1ull << G.wrap_min_work_log))
    return 0;
  if (make_cyclic_plan(P.p, P.m, P.n, P.k, d, j, P.elem_bytes, pc) != PM_OK) return 0;
  if (make_slice_plan(P.p, P.m, P.n, P.k, t, t, t - 1, t, P.elem_bytes, pt) != PM_OK) return 0;
  if (pc->ws_bytes > P.ws_bytes || pt->ws_bytes > P.ws_bytes) return 0;
  return j;
}

int wrap_log_of(const Plan& P) {
  Plan pc, pt;
  return wrap_log_plans(P, &pc, &pt);
}

int run_wrapped(const Plan& P, const void* A, const void* B, void* C, uint8_t* ws,
                uint64_t ws_bytes, hipStream_t s) {
  Plan Pc, Pt;
  const int j = wrap_log_plans(P, &Pc, &Pt);
  if (!j || Pc.ws_bytes > ws_bytes || Pt.ws_bytes > ws_bytes) return 0;
  const int d = P.d, Lp = 1 << j, t = 2 * d - 1 - Lp;
  const uint64_t eb = (uint64_t)P.elem_bytes;
  const int h = Lp - d + 1;
  const Plan both[2] = {Pc, Pt};
  int st = prepare_plans(both, 2, s);
  if (st != PM_OK) return st;
  st = run_product(Pc, A, B, C, ws, s, true);
  if (st != PM_OK) return st;
  const uint8_t* At = (const uint8_t*)A + eb * h * P.m * P.n;
  const uint8_t* Bt = (const uint8_t*)B + eb * h * P.n * P.k;
  uint8_t* Ct = (uint8_t*)C + eb * (uint64_t)Lp * P.m * P.k;
  st = run_product(Pt, At, Bt, Ct, ws, s, true);
  if (st != PM_OK) return st;
  const uint64_t mk = (uint64_t)P.m * P.k;
  KernelTimer kt(K_CRT, s);
  if (launch_unwrap(C, (uint64_t)t * mk, (uint64_t)Lp * mk, P.p, P.elem_bytes, s) !=
      hipSuccess)
    return PM_EDEVICE;
  return 1;
}

pm_status mul_common(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d, int elem_bytes,
                     const void* A, const void* B, void* C, void* ws, uint64_t ws_bytes,
                     void* stream) {
  Plan P;
  int st = make_plan(p, m, n, k, d, elem_bytes, &P);
  if (st != PM_OK) return (pm_status)st;
  if (P.mode == 1 && elem_bytes == 4 && d <= vdm_max_d() && vdm_eligible(p, m, n, k, d) &&
      ws_bytes >= P.ws_bytes)
    return pm_mul_vdm_u32((uint32_t)p, m, n, k, d, (const uint32_t*)A, (const uint32_t*)B,
                          (uint32_t*)C, ws, ws_bytes, stream);
  st = check_operands(P, A, B, C);
  if (st != PM_OK) return (pm_status)st;
  const uint64_t eb = (uint64_t)elem_bytes;
  st = check_workspace(ws, ws_bytes, P.ws_bytes, A, eb * d * m * n, B, eb * d * n * k, C,
                       eb * (2ull * d - 1) * m * k);
  if (st != PM_OK) return (pm_status)st;
  st = run_wrapped(P, A, B, C, (uint8_t*)ws, ws_bytes, (hipStream_t)stream);
  if (st == 1) return PM_OK;
  if (st != 0) return (pm_status)st;
  return (pm_status)run_product(P, A, B, C, (uint8_t*)ws, (hipStream_t)stream);
}

pm_status middle_common(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t da, int32_t db,
                        int32_t lo, int32_t len, int elem_bytes, const void* A, const void* B,
                        void* C, void* ws, uint64_t ws_bytes, void* stream) {
  Plan P;
  int st = make_slice_plan(p, m, n, k, da, db, lo, len, elem_bytes, &P);
  if (st != PM_OK) return (pm_status)st;
  st = check_operands(P, A, B, C);
  if (st != PM_OK) return (pm_status)st;
  const uint64_t eb = (uint64_t)elem_bytes;
  st = check_workspace(ws, ws_bytes, P.ws_bytes, A, eb * da * m * n, B, eb * db * n * k, C,
                       eb * (uint64_t)len * m * k);
  if (st != PM_OK) return (pm_status)st;
  return (pm_status)run_product(P, A, B, C, (uint8_t*)ws, (hipStream_t)stream);
}

}  // namespace

extern "C" {

pm_status pm_mul_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d, const uint32_t* A,
                     const uint32_t* B, uint32_t* C, void* workspace, uint64_t workspace_bytes,
                     void* stream) {
  return (pm_status)guarded([&] {
    return (int)mul_common(p, m, n, k, d, 4, A, B, C, workspace, workspace_bytes, stream);
  });
}

pm_status pm_mul_u64(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d, const uint64_t* A,
                     const uint64_t* B, uint64_t* C, void* workspace, uint64_t workspace_bytes,
                     void* stream) {
  return (pm_status)guarded([&] {
    return (int)mul_common(p, m, n, k, d, 8, A, B, C, workspace, workspace_bytes, stream);
  });
}

pm_status pm_mul_noalloc(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                         int32_t elem_bytes, const void* A, const void* B, void* C,
                         void* stream) {
  return (pm_status)guarded([&] {
    if (elem_bytes != 4 && elem_bytes != 8) return (int)PM_EINVAL;
    Plan P;
    int st = make_plan(p, m, n, k, d, elem_bytes, &P);
    if (st != PM_OK) return st;
    if (P.ws_bytes > kScratchWorkspaceBytes) return (int)PM_ESCRATCH;
    uint8_t* base = nullptr;
    st = noalloc_scratch(&base);
    if (st != PM_OK) return st;
    TablePool pool(kPoolStatic);
    return (int)mul_common(p, m, n, k, d, elem_bytes, A, B, C, base + kScratchTableBytes,
                           kScratchWorkspaceBytes, stream);
  });
}

pm_status pm_tables_bytes(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                          int32_t elem_bytes, uint64_t* out) {
  return (pm_status)guarded([&] {
    if (!out) return (int)PM_EINVAL;
    Plan P;
    int st = make_plan(p, m, n, k, d, elem_bytes, &P);
    if (st != PM_OK) return st;
    uint64_t b = (uint64_t)P.r * twiddle_table_bytes(P.logL, P.kn.split, P.kn.maxr);
    Plan pc, pt;
    if (wrap_log_plans(P, &pc, &pt))
      b += (uint64_t)pc.r * twiddle_table_bytes(pc.logL, pc.kn.split, pc.kn.maxr) +
           (uint64_t)pt.r * twiddle_table_bytes(pt.logL, pt.kn.split, pt.kn.maxr);
    if (P.mode == 1 && elem_bytes == 4 && d <= vdm_max_d() && vdm_eligible(p, m, n, k, d))
      b += vdm_table_bytes(d);
    *out = b;
    return (int)PM_OK;
  });
}

// ---- evaluation at 0 .. 2d-2 by Vandermonde products -------------------------

static uint64_t vdm_ws_bytes(int m, int n, int k, int d) {
  const uint64_t N = 2ull * d - 1;
  return align_up(4 * N * (uint64_t)m * n, 256) + align_up(4 * N * (uint64_t)n * k, 256) +
         align_up(4 * N * (uint64_t)m * k, 256);
}

static int vdm_check(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d) {
  if (m < 1 || n < 1 || k < 1 || d < 1) return PM_EINVAL;
  if (p < 2 || p >= (1ull << 31)) return PM_ERANGE;
  if (!is_prime_u64(p)) return PM_EINVAL;
  const uint64_t N = 2ull * d - 1;
  if (N > (uint64_t)p || N > (uint64_t)kGemmMaxK - 1 || n >= 4096) return PM_EUNSUPPORTED;
  const uint64_t lim = 1ull << 32;
  if (N * m * n >= lim || N * n * k >= lim || N * m * k >= lim) return PM_ERANGE;
  return PM_OK;
}

static void gemm_consts(uint32_t q, int K, GemmLaunch* g) {
  g->q = q;
  uint32_t inv = 1;  // q^{-1} mod 2^32 (q odd)
  for (int it = 0; it < 5; ++it) inv *= 2u - q * inv;
  g->qninv = 0u - inv;
  uint64_t w = (1ull << 32) % q;
  for (int s = 0; s < 7; ++s) {
    g->cs[s] = (uint32_t)w;
    w = (w << 8) % q;
  }
  g->bias = (uint64_t)q * 7ull * (uint64_t)K * 65536ull;
}

pm_status pm_vdm_workspace_bytes(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                                 uint64_t* out) {
  if (!out) return PM_EINVAL;
  const int st = vdm_check(p, m, n, k, d);
  if (st != PM_OK) return (pm_status)st;
  *out = vdm_ws_bytes(m, n, k, d);
  return PM_OK;
}

static pm_status vdm_impl(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                          const uint32_t* A, const uint32_t* B, uint32_t* C, void* workspace,
                          uint64_t workspace_bytes, void* stream);

pm_status pm_mul_vdm_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                         const uint32_t* A, const uint32_t* B, uint32_t* C, void* workspace,
                         uint64_t workspace_bytes, void* stream) {
  return (pm_status)guarded([&] {
    return (int)vdm_impl(p, m, n, k, d, A, B, C, workspace, workspace_bytes, stream);
  });
}

static pm_status vdm_impl(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                          const uint32_t* A, const uint32_t* B, uint32_t* C, void* workspace,
                          uint64_t workspace_bytes, void* stream) {
  int st = vdm_check(p, m, n, k, d);
  if (st != PM_OK) return (pm_status)st;
  if (p == 2) return PM_EUNSUPPORTED;  // the Montgomery epilogue needs q odd
  Plan P{};
  P.m = m; P.n = n; P.k = k; P.d = d; P.da = d; P.db = d; P.lo = 0; P.nout = 2 * d - 1;
  P.elem_bytes = 4;
  st = check_operands(P, A, B, C);
  if (st != PM_OK) return (pm_status)st;
  const uint64_t need = vdm_ws_bytes(m, n, k, d);
  st = check_workspace(workspace, workspace_bytes, need, A, 4ull * d * m * n, B,
                       4ull * d * n * k, C, 4ull * P.nout * m * k);
  if (st != PM_OK) return (pm_status)st;
  hipStream_t s = (hipStream_t)stream;
  const uint32_t *V = nullptr, *W = nullptr;
  st = prepare_vdm(p, d, s, &V, &W);
  if (st != PM_OK) return (pm_status)st;
  const int N = 2 * d - 1;
  uint8_t* ws = (uint8_t*)workspace;
  uint32_t* ahat = (uint32_t*)ws;
  uint32_t* bhat = (uint32_t*)(ws + align_up(4ull * N * m * n, 256));
  uint32_t* chat = (uint32_t*)(ws + align_up(4ull * N * m * n, 256) +
                               align_up(4ull * N * n * k, 256));
  {
    KernelTimer kt(K_VDM_EVAL, s);
    GemmLaunch g{};
    gemm_consts(p, d, &g);
    g.M = N; g.K = d; g.ldx = d; g.X = V;
    g.N = m * n; g.ldy = m * n; g.Y = A; g.ldz = m * n; g.Z = ahat;
    if (launch_gemm_modp(g, s) != hipSuccess) return PM_EDEVICE;
    g.N = n * k; g.ldy = n * k; g.Y = B; g.ldz = n * k; g.Z = bhat;
    if (launch_gemm_modp(g, s) != hipSuccess) return PM_EDEVICE;
  }
  {
    // one m x n by n x k product per point, no scaling (interpolation is W)
    PointwiseLaunch pw;
    memset(&pw, 0, sizeof pw);
    const Knobs kn = base_knobs();
    pw.m = m; pw.n = n; pw.k = k; pw.L = N;
    pw.small_lds = kn.pw_small_lds;
    pw.pipe = kn.pw_pipe;
    pw.ahat = ahat; pw.bhat = bhat; pw.chat = chat;
    pw.pc[0].q = p;
    pw.pc[0].linv = 1;
    pw.pc[0].linv_p = (uint32_t)((1ull << 32) / p);
    pw.pc[0].mu = ~0ull / p;
    GemmLaunch c{};
    gemm_consts(p, n, &c);
    for (int t = 0; t < 7; ++t) pw.cs[0][t] = c.cs[t];
    pw.bias[0] = c.bias;
    pw.qninv[0] = c.qninv;
    KernelTimer kt(K_POINTWISE, s);
    const int ok = choose_pointwise(m, n, k, kn.pointwise) == 1 ? launch_pointwise_mfma(pw, 1, s)
                                                                : launch_pointwise(pw, 1, s);
    if (ok != hipSuccess) return PM_EDEVICE;
  }
  {
    KernelTimer kt(K_VDM_INTERP, s);
    GemmLaunch g{};
    gemm_consts(p, N, &g);
    g.M = N; g.K = N; g.ldx = N; g.X = W;
    g.N = m * k; g.ldy = m * k; g.Y = chat; g.ldz = m * k; g.Z = C;
    if (launch_gemm_modp(g, s) != hipSuccess) return PM_EDEVICE;
  }
  return PM_OK;
}

// ---- evaluation at a geometric progression -------------------------------------

namespace {

// The four middle products of a geometric-progression product: the
// evaluations of A and B (chirp transforms), the chirp transform of the
// interpolation and the truncated product by Q.
struct GeoPlans {
  Plan a, b, i, q;
  uint64_t off_ra, off_rb, off_ah, off_bh, off_ch, off_y, off_s, off_w, total;
};

int geo_plans(uint64_t p, int m, int n, int k, int d, GeoPlans* G) {
  if (m < 1 || n < 1 || k < 1 || d < 1) return PM_EINVAL;
  if (p < 3 || p >= (1ull << 31)) return PM_ERANGE;
  if (!is_prime_u64(p)) return PM_EINVAL;
  if (n >= 4096) return PM_EUNSUPPORTED;  // the pointwise epilogue's bound
  const uint64_t N = 2ull * d - 1;
  if (N > p - 1) return PM_EUNSUPPORTED;  // no element of order >= N
  const int Ni = (int)N;
  int st = make_slice_plan(p, m * n, 1, 1, d, Ni + d - 1, d - 1, Ni, 4, &G->a);
  if (st != PM_OK) return st;
  st = make_slice_plan(p, n * k, 1, 1, d, Ni + d - 1, d - 1, Ni, 4, &G->b);
  if (st != PM_OK) return st;
  st = make_slice_plan(p, m * k, 1, 1, Ni, 2 * Ni - 1, Ni - 1, Ni, 4, &G->i);
  if (st != PM_OK) return st;
  st = make_slice_plan(p, m * k, 1, 1, Ni, Ni + 1, 0, Ni, 4, &G->q);
  if (st != PM_OK) return st;
  const uint64_t mn = (uint64_t)m * n, nk = (uint64_t)n * k, mk = (uint64_t)m * k;
  uint64_t off = 0;
  G->off_ra = off; off = align_up(off + 4 * d * mn, 256);
  G->off_rb = off; off = align_up(off + 4 * d * nk, 256);
  G->off_ah = off; off = align_up(off + 4 * N * mn, 256);
  G->off_bh = off; off = align_up(off + 4 * N * nk, 256);
  G->off_ch = off; off = align_up(off + 4 * N * mk, 256);
  G->off_y = off; off = align_up(off + 4 * N * mk, 256);
  G->off_s = off; off = align_up(off + 4 * N * mk, 256);
  G->off_w = off;
  off += std::max(std::max(G->a.ws_bytes, G->b.ws_bytes), std::max(G->i.ws_bytes, G->q.ws_bytes));
  G->total = align_up(off, 256);
  return PM_OK;
}

pm_status geo_impl(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d, const uint32_t* A,
                   const uint32_t* B, uint32_t* C, void* workspace, uint64_t workspace_bytes,
                   void* stream) {
  GeoPlans G;
  int st = geo_plans(p, m, n, k, d, &G);
  if (st != PM_OK) return (pm_status)st;
  Plan P{};
  P.m = m; P.n = n; P.k = k; P.d = d; P.da = d; P.db = d; P.lo = 0; P.nout = 2 * d - 1;
  P.elem_bytes = 4;
  st = check_operands(P, A, B, C);
  if (st != PM_OK) return (pm_status)st;
  st = check_workspace(workspace, workspace_bytes, G.total, A, 4ull * d * m * n, B,
                       4ull * d * n * k, C, 4ull * P.nout * m * k);
  if (st != PM_OK) return (pm_status)st;
  hipStream_t s = (hipStream_t)stream;
  GeoTables T;
  st = prepare_geo(p, d, s, &T);
  if (st != PM_OK) return (pm_status)st;
  const Plan all[4] = {G.a, G.b, G.i, G.q};
  st = prepare_plans(all, 4, s);
  if (st != PM_OK) return (pm_status)st;
  uint8_t* ws = (uint8_t*)workspace;
  uint32_t* ra = (uint32_t*)(ws + G.off_ra);
  uint32_t* rb = (uint32_t*)(ws + G.off_rb);
  uint32_t* ah = (uint32_t*)(ws + G.off_ah);
  uint32_t* bh = (uint32_t*)(ws + G.off_bh);
  uint32_t* ch = (uint32_t*)(ws + G.off_ch);
  uint32_t* y = (uint32_t*)(ws + G.off_y);
  uint32_t* sv = (uint32_t*)(ws + G.off_s);
  uint8_t* wp = ws + G.off_w;
  const uint32_t N = T.N;
  const uint64_t mn = (uint64_t)m * n, nk = (uint64_t)n * k, mk = (uint64_t)m * k;
  // evaluations: rows of A scaled by a^-C2(c) and reversed, the chirp
  // transform (coefficients d-1 .. d+N-2 of the product with a^C2(t)), the
  // values scaled by a^-C2(i)
  {
    KernelTimer kt(K_GEO, s);
    if (launch_geo_scale(A, ra, (uint32_t)d, mn, T.sneg, 1, p, s) != hipSuccess ||
        launch_geo_scale(B, rb, (uint32_t)d, nk, T.sneg, 1, p, s) != hipSuccess)
      return PM_EDEVICE;
  }
  st = run_product(G.a, ra, T.spos, ah, wp, s, true);
  if (st != PM_OK) return (pm_status)st;
  st = run_product(G.b, rb, T.spos, bh, wp, s, true);
  if (st != PM_OK) return (pm_status)st;
  {
    KernelTimer kt(K_GEO, s);
    if (launch_geo_scale(ah, ah, N, mn, T.sneg, 0, p, s) != hipSuccess ||
        launch_geo_scale(bh, bh, N, nk, T.sneg, 0, p, s) != hipSuccess)
      return PM_EDEVICE;
  }
  {
    // one m x n by n x k product per point, no scaling
    PointwiseLaunch pw;
    memset(&pw, 0, sizeof pw);
    const Knobs kn = base_knobs();
    pw.m = m; pw.n = n; pw.k = k; pw.L = (int)N;
    pw.small_lds = kn.pw_small_lds;
    pw.pipe = kn.pw_pipe;
    pw.ahat = ah; pw.bhat = bh; pw.chat = ch;
    pw.pc[0].q = p;
    pw.pc[0].linv = 1;
    pw.pc[0].linv_p = (uint32_t)((1ull << 32) / p);
    pw.pc[0].mu = ~0ull / p;
    GemmLaunch c{};
    gemm_consts(p, n, &c);
    for (int t = 0; t < 7; ++t) pw.cs[0][t] = c.cs[t];
    pw.bias[0] = c.bias;
    pw.qninv[0] = c.qninv;
    KernelTimer kt(K_POINTWISE, s);
    const int ok = choose_pointwise(m, n, k, kn.pointwise) == 1 ? launch_pointwise_mfma(pw, 1, s)
                                                                : launch_pointwise(pw, 1, s);
    if (ok != hipSuccess) return PM_EDEVICE;
  }
  // interpolation: values scaled by a^(C2(i) - i) / Q'(a^i) and reversed,
  // the chirp transform with a^-C2(t), scaled by -a^C2(k): the power series
  // S mod x^N; then C = (Q S) mod x^N
  {
    KernelTimer kt(K_GEO, s);
    if (launch_geo_scale(ch, y, N, mk, T.fc, 1, p, s) != hipSuccess) return PM_EDEVICE;
  }
  st = run_product(G.i, y, T.sneg, sv, wp, s, true);
  if (st != PM_OK) return (pm_status)st;
  {
    KernelTimer kt(K_GEO, s);
    if (launch_geo_scale(sv, sv, N, mk, T.nspos, 0, p, s) != hipSuccess) return PM_EDEVICE;
  }
  st = run_product(G.q, sv, T.q, C, wp, s, true);
  return (pm_status)st;
}

}  // namespace

extern "C" {

pm_status pm_geo_workspace_bytes(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                                 uint64_t* out) {
  return (pm_status)guarded([&] {
    if (!out) return (int)PM_EINVAL;
    GeoPlans G;
    const int st = geo_plans(p, m, n, k, d, &G);
    if (st != PM_OK) return st;
    *out = G.total;
    return (int)PM_OK;
  });
}

pm_status pm_mul_geo_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                         const uint32_t* A, const uint32_t* B, uint32_t* C, void* workspace,
                         uint64_t workspace_bytes, void* stream) {
  return (pm_status)guarded([&] {
    return (int)geo_impl(p, m, n, k, d, A, B, C, workspace, workspace_bytes, stream);
  });
}

}  // extern "C"

pm_status pm_middle_plan(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t da, int32_t db,
                         int32_t lo, int32_t len, int32_t elem_bytes, pm_plan_info* out) {
  return (pm_status)guarded([&] {
    if (!out) return (int)PM_EINVAL;
    Plan P;
    int st = make_slice_plan(p, m, n, k, da, db, lo, len, elem_bytes, &P);
    if (st != PM_OK) return st;
    fill_plan_info(P, out);
    return (int)PM_OK;
  });
}

pm_status pm_middle_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t da, int32_t db,
                        int32_t lo, int32_t len, const uint32_t* A, const uint32_t* B,
                        uint32_t* C, void* workspace, uint64_t workspace_bytes, void* stream) {
  return (pm_status)guarded([&] {
    return (int)middle_common(p, m, n, k, da, db, lo, len, 4, A, B, C, workspace,
                              workspace_bytes, stream);
  });
}

pm_status pm_middle_u64(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t da, int32_t db,
                        int32_t lo, int32_t len, const uint64_t* A, const uint64_t* B,
                        uint64_t* C, void* workspace, uint64_t workspace_bytes, void* stream) {
  return (pm_status)guarded([&] {
    return (int)middle_common(p, m, n, k, da, db, lo, len, 8, A, B, C, workspace,
                              workspace_bytes, stream);
  });
}

pm_status pm_neg_mod(uint64_t p, const void* X, void* Y, uint64_t count, int32_t elem_bytes,
                     void* stream) {
  if (!X || !Y || (elem_bytes != 4 && elem_bytes != 8)) return PM_EINVAL;
  if (p < 2) return PM_EINVAL;
  if ((elem_bytes == 4 && p > 0xFFFFFFFFull) || (elem_bytes == 8 && p >= (1ull << 62)))
    return PM_ERANGE;
  if (((uintptr_t)X | (uintptr_t)Y) & (uintptr_t)(elem_bytes - 1)) return PM_EINVAL;
  const uint64_t bytes = count * (uint64_t)elem_bytes;
  if (count && X != Y && overlap(X, bytes, Y, bytes)) return PM_EINVAL;
  if (!count) return PM_OK;
  KernelTimer kt(K_CRT, (hipStream_t)stream);
  return launch_neg_mod(p, X, Y, count, elem_bytes, (hipStream_t)stream) == hipSuccess
             ? PM_OK
             : PM_EDEVICE;
}

pm_status pm_probe_valu(uint32_t blocks, uint32_t iters, void* out, void* stream) {
  if (!out || blocks == 0 || blocks > (1u << 20) || iters == 0 || ((uintptr_t)out & 3))
    return PM_EINVAL;
  return launch_probe_mulhi((uint32_t*)out, blocks, iters, 0x9E3779B1u, (hipStream_t)stream) ==
                 hipSuccess
             ? PM_OK
             : PM_EDEVICE;
}

pm_status pm_check_residues(uint64_t p, const void* X, uint64_t count, int32_t elem_bytes,
                            uint64_t* n_bad, void* workspace, void* stream) {
  if (!X || !n_bad || !workspace || (elem_bytes != 4 && elem_bytes != 8)) return PM_EINVAL;
  if (((uintptr_t)X & (elem_bytes - 1)) || ((uintptr_t)workspace & 7)) return PM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long* counter = (unsigned long long*)workspace;
  // The counter is cleared by a kernel-free copy of a host zero (no memset
  // node, so the sequence can be graph-captured).
  static const unsigned long long zero = 0;
  if (hipMemcpyAsync(counter, &zero, sizeof zero, hipMemcpyHostToDevice, s) != hipSuccess)
    return PM_EDEVICE;
  if (count && launch_check_residues(p, X, count, elem_bytes, counter, s) != hipSuccess)
    return PM_EDEVICE;
  unsigned long long h = 0;
  if (hipMemcpyAsync(&h, counter, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess)
    return PM_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return PM_EDEVICE;
  *n_bad = h;
  return PM_OK;
}

pm_status pm_sync(void* stream) {
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PM_EDEVICE;
  if (hipGetLastError() != hipSuccess) return PM_EDEVICE;
  return PM_OK;
}

}  // extern "C"

// ---- operand evaluations (multiplier precomputation) -----------------------------

namespace {

// Plan of a product in which X is the left (role 0) or right (role 1) operand.
int eval_plan(uint64_t p, int32_t role, int32_t rows, int32_t cols, int32_t d, int eb, Plan* P) {
  if (role != 0 && role != 1) return PM_EINVAL;
  return role == 0 ? make_plan(p, rows, cols, 1, d, eb, P) : make_plan(p, 1, rows, cols, d, eb, P);
}

uint64_t eval_prime_stride_bytes(const Plan& P, int32_t rows, int32_t cols) {
  return align_up(4ull * ((uint64_t)1 << P.logL) * (uint64_t)rows * cols, 256);
}

pm_status eval_common(uint64_t p, int32_t role, int32_t rows, int32_t cols, int32_t d, int eb,
                      const void* X, void* Xe, uint64_t xe_bytes, void* stream) {
  Plan P;
  int st = eval_plan(p, role, rows, cols, d, eb, &P);
  if (st != PM_OK) return (pm_status)st;
  if (!X || !Xe || ((uintptr_t)X & 15) || ((uintptr_t)Xe & 255)) return PM_EINVAL;
  const uint64_t need = eval_prime_stride_bytes(P, rows, cols) * P.r;
  if (xe_bytes < need) return PM_EWORKSPACE;
  if (overlap(X, (uint64_t)eb * d * rows * cols, Xe, need)) return PM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  st = prepare_plans(&P, 1, s);
  if (st != PM_OK) return (pm_status)st;
  PrimeConst pc[kMaxPrimes];
  for (int i = 0; i < P.r; ++i) {
    st = prime_const(TwKey{P.q[i], P.logL, P.kn.split, P.kn.maxr}, &pc[i]);
    if (st != PM_OK) return (pm_status)st;
  }
  // Evaluations come out in bit-reversed point order whatever the pass
  // structure, so a product planned with other knobs can consume them.
  NttLaunch a;
  memset(&a, 0, sizeof a);
  fill_ntt_launch(&a, P.logL, rows * cols, d, eb, false, false, P.kn);
  a.lazy = lazy_ok(P);
  for (int i = 0; i < P.r; ++i) a.pc[i] = pc[i];
  a.in = X;
  a.out = Xe;
  a.in_prime_stride = 0;
  a.out_prime_stride = eval_prime_stride_bytes(P, rows, cols) / 4;
  KernelTimer kt(K_NTT_FWD, s);
  if (launch_ntt_fwd(a, eb, P.mode == 1, P.r, s) != hipSuccess) return PM_EDEVICE;
  return PM_OK;
}

}  // namespace

extern "C" {

pm_status pm_eval_bytes(uint64_t p, int32_t role, int32_t rows, int32_t cols, int32_t d,
                        int32_t elem_bytes, uint64_t* out) {
  return (pm_status)guarded([&] {
    if (!out) return (int)PM_EINVAL;
    Plan P;
    int st = eval_plan(p, role, rows, cols, d, elem_bytes, &P);
    if (st != PM_OK) return st;
    *out = eval_prime_stride_bytes(P, rows, cols) * P.r;
    return (int)PM_OK;
  });
}

pm_status pm_eval_u32(uint32_t p, int32_t role, int32_t rows, int32_t cols, int32_t d,
                      const uint32_t* X, void* X_eval, uint64_t eval_bytes, void* stream) {
  return (pm_status)guarded([&] {
    return (int)eval_common(p, role, rows, cols, d, 4, X, X_eval, eval_bytes, stream);
  });
}

pm_status pm_eval_u64(uint64_t p, int32_t role, int32_t rows, int32_t cols, int32_t d,
                      const uint64_t* X, void* X_eval, uint64_t eval_bytes, void* stream) {
  return (pm_status)guarded([&] {
    return (int)eval_common(p, role, rows, cols, d, 8, X, X_eval, eval_bytes, stream);
  });
}

}  // extern "C"

// ---- batched products ---------------------------------------------------------

namespace {

// Segments a product contributes to the six phases (see pm_batch.h).
int count_segments(const Plan& P) {
  const int split = P.kn.split ? 1 : 0;
  return 2 * P.r                 // forward first pass / unsplit forward
         + 2 * P.r * split       // forward blocks
         + P.r                   // pointwise
         + P.r * split           // inverse blocks
         + P.r                   // inverse last pass / unsplit inverse
         + (P.mode == 1 ? 1 : 0);
}

struct BatchLayout {
  uint64_t prod_off;   // ProductLaunches[count]
  uint64_t seg_off;    // BatchSeg[total segments]
  uint64_t total;
  uint64_t nseg;
};

// Workspace layout of a batch whose plans are made: per-product workspaces,
// then the product descriptors and the segment table.
void layout_batch(const std::vector<Plan>& plans, std::vector<uint64_t>& offs, BatchLayout* lay) {
  const int count = (int)plans.size();
  offs.resize(count);
  uint64_t off = 0, nseg = 0;
  for (int32_t i = 0; i < count; ++i) {
    offs[i] = off;
    off = align_up(off + plans[i].ws_bytes, 256);
    nseg += count_segments(plans[i]);
  }
  lay->prod_off = off;
  off = align_up(off + sizeof(ProductLaunches) * (uint64_t)count, 256);
  lay->seg_off = off;
  off = align_up(off + sizeof(BatchSeg) * nseg, 256);
  lay->total = off;
  lay->nseg = nseg;
}

int plan_batch(uint64_t p, int32_t count, const pm_product* prods, int32_t elem_bytes,
               std::vector<Plan>& plans, std::vector<uint64_t>& offs, BatchLayout* lay) {
  alloc_point();
  plans.resize(count);
  for (int32_t i = 0; i < count; ++i) {
    const pm_product& pr = prods[i];
    int st = make_plan(p, pr.m, pr.n, pr.k, pr.d, elem_bytes, &plans[i]);
    if (st != PM_OK) return st;
  }
  layout_batch(plans, offs, lay);
  return PM_OK;
}

// Corrections of the wrapped products of a batch (as in run_wrapped).
struct UnwrapJob {
  void* C;
  uint64_t count, off, p;
  int elem_bytes;
};

// The entries a batch runs: a whole product that pm_mul computes in the
// wrapped form (and that carries no precomputed evaluations, which are at
// the plain length) becomes two, the cyclic product into C and the product
// of the tops into C's rows 2^j .., plus a correction after the batch;
// other products stay as they are.
void expand_wrapped(const std::vector<Plan>& plans, const pm_product* prods, int eb,
                    std::vector<Plan>* xplans, std::vector<pm_product>* xprods,
                    std::vector<UnwrapJob>* jobs) {
  for (size_t i = 0; i < plans.size(); ++i) {
    const Plan& P = plans[i];
    const pm_product& pr = prods[i];
    Plan Pc, Pt;
    const int j = (pr.A_eval || pr.B_eval) ? 0 : wrap_log_plans(P, &Pc, &Pt);
    if (!j) {
      xplans->push_back(P);
      xprods->push_back(pr);
      continue;
    }
    const int d = P.d, Lp = 1 << j, t = 2 * d - 1 - Lp, h = Lp - d + 1;
    const uint64_t mk = (uint64_t)P.m * P.k;
    xplans->push_back(Pc);
    xprods->push_back(pm_product{P.m, P.n, P.k, d, pr.A, pr.B, pr.C, nullptr, nullptr});
    xplans->push_back(Pt);
    xprods->push_back(pm_product{P.m, P.n, P.k, 0,
                                 (const uint8_t*)pr.A + (uint64_t)eb * h * P.m * P.n,
                                 (const uint8_t*)pr.B + (uint64_t)eb * h * P.n * P.k,
                                 (uint8_t*)pr.C + (uint64_t)eb * Lp * mk, nullptr, nullptr});
    jobs->push_back(UnwrapJob{pr.C, (uint64_t)t * mk, (uint64_t)Lp * mk, P.p, eb});
  }
}

// Plans of a batch of coefficient windows (pm_window_product), with the
// products re-expressed as pm_product (no precomputed evaluations) for the
// shared launch code.
int plan_window_batch(uint64_t p, int32_t count, const pm_window_product* wins,
                      int32_t elem_bytes, std::vector<Plan>& plans, std::vector<uint64_t>& offs,
                      BatchLayout* lay, std::vector<pm_product>* prods) {
  alloc_point();
  plans.resize(count);
  if (prods) prods->resize(count);
  for (int32_t i = 0; i < count; ++i) {
    const pm_window_product& w = wins[i];
    int st = make_slice_plan(p, w.m, w.n, w.k, w.da, w.db, w.lo, w.len, elem_bytes, &plans[i]);
    if (st != PM_OK) return st;
    if (prods) (*prods)[i] = pm_product{w.m, w.n, w.k, 0, w.A, w.B, w.C, nullptr, nullptr};
  }
  layout_batch(plans, offs, lay);
  return PM_OK;
}

struct HostSeg {
  BatchSeg g;
  uint32_t count;
  double cost;     // per tile
  uint32_t lds;    // bytes of LDS a tile needs
};

// LDS classes: tiles of one phase are launched in groups so that small tiles
// are not held to the occupancy of the largest.  Class c holds footprints up
// to 160 KiB / n_c (rounded down to 256 bytes) for n_c = 10, 8, 7, 6, 5, 4,
// 3, 2, 1 workgroups per CU.
constexpr int kLdsClasses = 9;
static const uint32_t kLdsClassMax[kLdsClasses] = {16384, 20480, 23296, 27136, 32768,
                                                   40960, 54528, 81920, 163840};
int lds_class(uint32_t bytes) {
  for (int c = 0; c < kLdsClasses; ++c)
    if (bytes <= kLdsClassMax[c]) return c;
  return kLdsClasses - 1;
}

size_t ntt_lds_bytes(const NttLaunch& a) { return 4 * (size_t)a.lds_stride << a.eb_log; }

// Build the segments of one product into the per-phase lists; track LDS needs.
void product_segments(uint32_t idx, const Plan& P, const ProductLaunches& L, bool a_given,
                      bool b_given, std::vector<HostSeg>* ph, size_t* lds) {
  auto add = [&](int phase, uint16_t kind, uint16_t op, uint16_t prime, uint32_t nx,
                 uint32_t count, double cost, size_t need, uint16_t zpts) {
    HostSeg h;
    memset(&h, 0, sizeof h);
    h.g.prod = idx; h.g.nx = nx; h.g.kind = kind; h.g.op = op; h.g.prime = prime;
    h.g.zpts = zpts;
    h.count = count;
    h.cost = cost;
    h.lds = (uint32_t)need;
    ph[phase].push_back(h);
    (void)lds;
  };
  const uint32_t L_ = 1u << P.logL;
  for (int op = 0; op < 2; ++op) {
    if ((op == 0 && a_given) || (op == 1 && b_given)) continue;
    const NttLaunch& a = L.f[op];
    const uint32_t EB = 1u << a.eb_log;
    const uint32_t neb = ((uint32_t)a.E + EB - 1) / EB;
    for (int q = 0; q < P.r; ++q) {
      if (a.split) {
        const uint32_t items = col_items(a);
        const uint32_t n0 = (items + kColChunk - 1) / kColChunk;
        add(0, BK_COL_FWD, op, q, n0, n0, (double)(items < kColChunk ? items : kColChunk) *
                                              a.col_vec * (1 << a.split), 0, 0);
        add(1, BK_BLOCK_FWD, op, q, neb, neb * a.keep,
            (double)EB * (1u << a.blk_log) * (a.logL - a.split), block_lds_bytes(a), 0);
      } else {
        add(0, BK_FWD_LDS, op, q, neb, neb, (double)EB * L_ * (P.logL + 1), ntt_lds_bytes(a), 0);
      }
    }
  }
  {
    // points per tile: about batch_pw_work (default 8192) MACs of work;
    // pipelined tiles (limb planes above the 256-thread limit): about
    // batch_pw_pipe_pts (default 16) points each, so that a workgroup's loads
    // run ahead of its products
    const GlobalKnobs G = global_knobs();
    const double pw_work = (double)G.batch_pw_work;
    const double pipe_pts = (double)G.batch_pw_pipe_pts;
    const double mnk = (double)P.m * P.n * P.k;
    size_t need = 0;
    if (L.pointwise == 1) need = pointwise_mfma_lds(P.m, P.n, P.k);
    else if (L.pw_staged) need = 4ull * ((uint64_t)P.m * P.n + (uint64_t)P.n * P.k);
    const int pipe = L.pointwise == 1 && need > (size_t)base_knobs().pw_small_lds
                         ? pointwise_pipe_variant(P.m, P.n, P.k, P.kn.pw_pipe) : 0;
    uint32_t z = (uint32_t)(pw_work / mnk);
    if (pipe && z < (uint32_t)pipe_pts) z = (uint32_t)pipe_pts;
    if (z < 1) z = 1;
    const uint32_t npts = (uint32_t)P.npts;
    if (z > npts) z = npts;
    if (z > 65535) z = 65535;
    const uint32_t nt = (npts + z - 1) / z;
    for (int q = 0; q < P.r; ++q)
      add(pipe == 2 ? 6 : 2, BK_PW, pipe == 1 ? 1 : 0, q, nt, nt, z * mnk, need, (uint16_t)z);
  }
  {
    const NttLaunch& a = L.inv;
    const uint32_t EB = 1u << a.eb_log;
    const uint32_t neb = ((uint32_t)a.E + EB - 1) / EB;
    for (int q = 0; q < P.r; ++q) {
      if (a.split) {
        add(3, BK_BLOCK_INV, 0, q, neb, neb * a.keep,
            (double)EB * (1u << a.blk_log) * (a.logL - a.split), block_lds_bytes(a), 0);
        const uint32_t items = col_items(a);
        const uint32_t n0 = (items + kColChunk - 1) / kColChunk;
        add(4, BK_COL_INV, 0, q, n0, n0, (double)(items < kColChunk ? items : kColChunk) *
                                             a.col_vec * (1 << a.split), 0, 0);
      } else {
        add(4, BK_INV_LDS, 0, q, neb, neb, (double)EB * L_ * (P.logL + 1), ntt_lds_bytes(a), 0);
      }
    }
  }
  if (P.mode == 1) {
    const uint32_t n = (uint32_t)((L.crt.count + kCrtChunk - 1) / kCrtChunk);
    add(5, BK_CRT, 0, 0, n, n, (double)kCrtChunk * P.r, 0, 0);
  }
}

// Host side of a phase-launched batch: descriptors and segment tables (to be
// copied to ws + lay.prod_off) and the launch groups.
struct BatchGroup {
  int phase;
  uint64_t first_seg, nseg, tiles;
  uint32_t lds;
};
struct BatchBuild {
  std::vector<uint8_t> host;
  std::vector<BatchGroup> groups;
};

int build_batch(const std::vector<Plan>& plans, const std::vector<uint64_t>& offs,
                const BatchLayout& lay, const pm_product* prods, uint8_t* ws, BatchBuild* B) {
  const int count = (int)plans.size();
  B->host.assign(lay.total - lay.prod_off, 0);
  B->groups.clear();
  ProductLaunches* hp = (ProductLaunches*)B->host.data();
  std::vector<HostSeg> ph[kBatchPhases];
  size_t lds[kBatchPhases] = {};  // unused: LDS is tracked per segment
  for (int i = 0; i < count; ++i) {
    const Plan& P = plans[i];
    // the phase kernels run column passes of 2 to 4 stages (run_batch gives
    // products planned with 5 a 4-stage pass or the single-product kernels)
    if (P.kn.split > 4) return PM_EUNSUPPORTED;
    int st = fill_product_launches(P, prods[i].A, prods[i].B, prods[i].C, ws + offs[i], &hp[i],
                                   true);
    if (st != PM_OK) return st;
    // the phase kernels run column items of at most two entries (register
    // budget: two workgroups per CU)
    for (NttLaunch* a : {&hp[i].f[0], &hp[i].f[1], &hp[i].inv})
      if (a->col_vec > 2) a->col_vec = 2;
    // given evaluations replace the forward transforms of that operand
    if (prods[i].A_eval) {
      hp[i].pw.ahat = (const uint32_t*)prods[i].A_eval;
      hp[i].pw.a_prime_stride = eval_prime_stride_bytes(P, P.m, P.n) / 4;
    }
    if (prods[i].B_eval) {
      hp[i].pw.bhat = (const uint32_t*)prods[i].B_eval;
      hp[i].pw.b_prime_stride = eval_prime_stride_bytes(P, P.n, P.k) / 4;
    }
    product_segments((uint32_t)i, P, hp[i], prods[i].A_eval != nullptr,
                     prods[i].B_eval != nullptr, ph, lds);
  }
  // Per phase and LDS class: largest tiles first, then prefix sums of tile
  // counts; one launch per non-empty (phase, class).
  BatchSeg* hs = (BatchSeg*)(B->host.data() + (lay.seg_off - lay.prod_off));
  uint64_t seg_base = 0;
  for (int fo = 0; fo < kBatchPhases; ++fo) {
    const int f = kBatchPhaseOrder[fo];
    std::vector<HostSeg> cls[kLdsClasses];
    for (auto& h : ph[f]) cls[lds_class(h.lds)].push_back(h);
    for (int c = 0; c < kLdsClasses; ++c) {
      if (cls[c].empty()) continue;
      std::stable_sort(cls[c].begin(), cls[c].end(),
                       [](const HostSeg& a, const HostSeg& b) { return a.cost > b.cost; });
      BatchGroup G{f, seg_base, cls[c].size(), 0, 0};
      for (auto& h : cls[c]) {
        h.g.first = (uint32_t)G.tiles;
        G.tiles += h.count;
        if (h.lds > G.lds) G.lds = h.lds;
        hs[seg_base++] = h.g;
      }
      if (G.tiles > 0x7fffffffull) return PM_ERANGE;
      B->groups.push_back(G);
    }
  }
  if (seg_base > lay.nseg) return PM_EINVAL;
  return PM_OK;
}

int enqueue_batch(const BatchBuild& B, const void* host_src, const BatchLayout& lay, uint8_t* ws,
                  hipStream_t s) {
  if (hipMemcpyAsync(ws + lay.prod_off, host_src, B.host.size(), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return PM_EDEVICE;
  const ProductLaunches* dprods = (const ProductLaunches*)(ws + lay.prod_off);
  const BatchSeg* dsegs = (const BatchSeg*)(ws + lay.seg_off);
  static const int kind_of_phase[kBatchPhases] = {K_NTT_FWD, K_NTT_FWD, K_POINTWISE, K_NTT_INV,
                                                  K_NTT_INV, K_CRT,     K_POINTWISE};
  KernelTimer kt(K_BATCHED, s, true);
  for (const BatchGroup& G : B.groups) {
    KernelTimer kp(kind_of_phase[G.phase], s);
    if (launch_batch_phase(G.phase, dprods, dsegs + G.first_seg, (int)G.nseg,
                           (uint32_t)G.tiles, G.lds, s) != hipSuccess)
      return PM_EDEVICE;
  }
  return PM_OK;
}

// Small batches: per-product launches with their parameters in kernel
// arguments (no descriptor upload, no phase tables).
int run_direct(const std::vector<Plan>& plans, const std::vector<uint64_t>& offs,
               const pm_product* prods, uint8_t* ws, hipStream_t s) {
  for (size_t i = 0; i < plans.size(); ++i) {
    const Plan& P = plans[i];
    ProductLaunches L;
    int st = fill_product_launches(P, prods[i].A, prods[i].B, prods[i].C, ws + offs[i], &L);
    if (st != PM_OK) return st;
    if (prods[i].A_eval) {
      L.pw.ahat = (const uint32_t*)prods[i].A_eval;
      L.pw.a_prime_stride = eval_prime_stride_bytes(P, P.m, P.n) / 4;
    }
    if (prods[i].B_eval) {
      L.pw.bhat = (const uint32_t*)prods[i].B_eval;
      L.pw.b_prime_stride = eval_prime_stride_bytes(P, P.n, P.k) / 4;
    }
    const bool skip[2] = {prods[i].A_eval != nullptr, prods[i].B_eval != nullptr};
    st = launch_product(P, L, skip, s);
    if (st != PM_OK) return st;
  }
  return PM_OK;
}

// ---- graph cache: a batch that repeats (same products, pointers, workspace)
// is captured once into a HIP graph and replayed.  The first occurrence runs
// eagerly, so tables and kernel attributes exist before any capture; the
// second is captured; later ones replay.  Each entry owns the pinned host
// copy of its descriptors that its memcpy node reads.
struct GraphEntry {
  std::vector<uint8_t> sig;
  int seen = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* pinned = nullptr;
  hipStream_t last = nullptr;
  uint64_t tick = 0;
  uint64_t epoch = 0;  // cache_epoch() when the entry was made
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
uint64_t g_tick = 0;
constexpr size_t kGraphCacheMax = 16;
// Graphs embed table pointers and launch shapes: a table reset or a new
// tuning table makes them stale.
uint64_t cache_epoch() { return (tables_epoch() << 32) ^ tune_epoch(); }

void free_entry(GraphEntry& e) {
  if (e.last) (void)hipStreamSynchronize(e.last);  // a replay may still read `pinned`
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  if (e.pinned) (void)hipHostFree(e.pinned);
  e = GraphEntry();
}

// One non-blocking capture stream per device, default priority, kept for
// the life of the process.
hipStream_t capture_stream(int dev) {
  static hipStream_t streams[64] = {};
  if (dev < 0 || dev >= 64) return nullptr;
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

std::vector<uint8_t> batch_signature(uint64_t p, int eb, const pm_product* prods,
                                     const std::vector<Plan>& plans, const void* ws,
                                     uint64_t ws_bytes, int dev) {
  const int count = (int)plans.size();
  std::vector<uint8_t> sig(sizeof(uint64_t) * 3 + sizeof(int) * 2 +
                           (sizeof(pm_product) + 4 * sizeof(int)) * count);
  uint8_t* o = sig.data();
  auto put = [&](const void* x, size_t n) { memcpy(o, x, n); o += n; };
  const uint64_t w = (uint64_t)(uintptr_t)ws;
  put(&p, 8); put(&w, 8); put(&ws_bytes, 8); put(&eb, sizeof eb); put(&dev, sizeof dev);
  put(prods, sizeof(pm_product) * count);
  for (const Plan& P : plans) {  // coefficient windows (whole products: d, d, 0, 2d-1)
    const int win[4] = {P.da, P.db, P.lo, P.nout};
    put(win, sizeof win);
  }
  return sig;
}

int run_batch_phases(uint64_t p, int eb, const std::vector<Plan>& plans,
                     const std::vector<uint64_t>& offs, const BatchLayout& lay,
                     const pm_product* prods, uint8_t* ws, uint64_t ws_bytes, hipStream_t s);

// log2 of a product's transform work, (mn + nk + mk) points primes.
double work_log2(const Plan& P) {
  const double e = (double)P.m * P.n + (double)P.n * P.k + (double)P.m * P.k;
  return std::log2(e * (double)P.npts * (double)P.r);
}

int run_batch(uint64_t p, int eb, const std::vector<Plan>& plans,
              const std::vector<uint64_t>& offs, const BatchLayout& lay, const pm_product* prods,
              uint8_t* ws, uint64_t ws_bytes, hipStream_t s) {
  const int count = (int)plans.size();
  // Global knobs: batch_direct_max (default 2) is the largest batch launched
  // per product; batch_single_min_log (see below).
  const GlobalKnobs G = global_knobs();
  int st = prepare_plans(plans.data(), plans.size(), s);
  if (st != PM_OK) return st;
  if (count <= G.batch_direct_max) return run_direct(plans, offs, prods, ws, s);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    // The caller is capturing a graph of its own: the phase launches would
    // record a copy of descriptors from host memory that this call cannot
    // keep alive for the graph's lifetime, so the products are launched one
    // by one with their parameters in kernel arguments (same results).
    return run_direct(plans, offs, prods, ws, s);
  }
  // Products whose transforms fill the device on their own, (mn + nk + mk)
  // points primes >= 2^batch_single_min_log, gain nothing from sharing
  // launches and run faster on the single-product kernels (launch shapes
  // tuned per shape, both operands per launch): they are launched that way,
  // ahead of the phase launches of the others (0: never; default 25, the
  // best of 18..30 on 512 products of the batched shape rule: 77 products
  // as single launches, 56.8 -> 55.5 ms per call; more singles lose to the
  // shared launches, 62.6 ms at 18).
  //
  // The phase kernels run column passes of at most 4 stages: a product whose
  // plan has 5 and that stays in the phases runs a 4-stage first pass there
  // (same points and workspace, another pass structure).
  std::vector<Plan> bp, rp;
  std::vector<uint64_t> bo, ro;
  std::vector<pm_product> bpr, rpr;
  bool clamped = false;
  for (int i = 0; i < count; ++i) {
    const bool big = G.batch_single_min_log > 0 &&
                     work_log2(plans[i]) >= (double)G.batch_single_min_log;
    Plan q = plans[i];
    if (!big && q.kn.split > 4) {
      q.kn.split = 4;
      q.keep = q.trunc ? 3 << 2 : 1 << 4;
      clamped = true;
    }
    (big ? bp : rp).push_back(q);
    (big ? bo : ro).push_back(offs[i]);
    (big ? bpr : rpr).push_back(prods[i]);
  }
  if (clamped) {
    st = prepare_plans(rp.data(), rp.size(), s);
    if (st != PM_OK) return st;
  }
  if (!bp.empty()) {
    st = run_direct(bp, bo, bpr.data(), ws, s);
    if (st != PM_OK || rp.empty()) return st;
    if ((int)rp.size() <= G.batch_direct_max) return run_direct(rp, ro, rpr.data(), ws, s);
  }
  return run_batch_phases(p, eb, rp, ro, lay, rpr.data(), ws, ws_bytes, s);
}

// The phase launches of a batch (graph replay from the second occurrence of
// the same batch; global knob batch_graph 0 turns replay off).
int run_batch_phases(uint64_t p, int eb, const std::vector<Plan>& plans,
                     const std::vector<uint64_t>& offs, const BatchLayout& lay,
                     const pm_product* prods, uint8_t* ws, uint64_t ws_bytes, hipStream_t s) {
  const GlobalKnobs G = global_knobs();
  const bool use_graphs = G.batch_graph != 0;
  int st = PM_OK;
  if (!use_graphs) {
    BatchBuild B;
    st = build_batch(plans, offs, lay, prods, ws, &B);
    if (st != PM_OK) return st;
    return enqueue_batch(B, B.host.data(), lay, ws, s);
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PM_EDEVICE;
  std::vector<uint8_t> sig = batch_signature(p, eb, prods, plans, ws, ws_bytes, dev);
  std::lock_guard<std::mutex> lock(g_graph_mu);
  GraphEntry* e = nullptr;
  for (auto& g : g_graphs)
    if (g.sig == sig) { e = &g; break; }
  if (e && e->epoch != cache_epoch()) {
    // tables were reset since this graph was captured: its table pointers
    // are stale
    free_entry(*e);
    g_graphs.erase(g_graphs.begin() + (e - g_graphs.data()));
    e = nullptr;
  }
  if (e && e->exec) {
    e->tick = ++g_tick;
    e->last = s;
    KernelTimer kt(K_BATCHED, s, true);
    return hipGraphLaunch(e->exec, s) == hipSuccess ? PM_OK : PM_EDEVICE;
  }
  BatchBuild B;
  st = build_batch(plans, offs, lay, prods, ws, &B);
  if (st != PM_OK) return st;
  if (!e) {
    // first occurrence: remember the signature, run eagerly
    if (g_graphs.size() >= kGraphCacheMax) {
      auto lru = std::min_element(g_graphs.begin(), g_graphs.end(),
                                  [](const GraphEntry& a, const GraphEntry& b) {
                                    return a.tick < b.tick;
                                  });
      free_entry(*lru);
      g_graphs.erase(lru);
    }
    GraphEntry ne;
    ne.sig = std::move(sig);
    ne.seen = 1;
    ne.epoch = cache_epoch();
    ne.tick = ++g_tick;
    g_graphs.push_back(std::move(ne));
    return enqueue_batch(B, B.host.data(), lay, ws, s);
  }
  // second occurrence: capture on a library stream (the caller's may be the
  // legacy default stream, which cannot be captured), instantiate, and
  // launch the graph on the caller's stream.
  hipStream_t cap = capture_stream(dev);
  if (!cap || hipHostMalloc(&e->pinned, B.host.size(), hipHostMallocDefault) != hipSuccess) {
    e->pinned = nullptr;
    (void)hipGetLastError();
    return enqueue_batch(B, B.host.data(), lay, ws, s);
  }
  memcpy(e->pinned, B.host.data(), B.host.size());
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(e->pinned);
    e->pinned = nullptr;
    return enqueue_batch(B, B.host.data(), lay, ws, s);
  }
  st = enqueue_batch(B, e->pinned, lay, ws, cap);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(cap, &graph);
  if (st != PM_OK || ce != hipSuccess || !graph) {
    // capture failed: nothing was run; clear the error and run eagerly
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    (void)hipHostFree(e->pinned);
    e->pinned = nullptr;
    return enqueue_batch(B, B.host.data(), lay, ws, s);
  }
  e->graph = graph;
  if (hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    e->exec = nullptr;
    (void)hipGraphDestroy(graph);
    e->graph = nullptr;
    (void)hipHostFree(e->pinned);
    e->pinned = nullptr;
    return enqueue_batch(B, B.host.data(), lay, ws, s);
  }
  e->tick = ++g_tick;
  e->last = s;
  KernelTimer kt(K_BATCHED, s, true);
  return hipGraphLaunch(e->exec, s) == hipSuccess ? PM_OK : PM_EDEVICE;
}

}  // namespace

extern "C" {

pm_status pm_batched_workspace_bytes(uint64_t p, int32_t count, const pm_product* prods,
                                     int32_t elem_bytes, uint64_t* out) {
  if (!out || count < 0 || (count > 0 && !prods)) return PM_EINVAL;
  try {
    std::vector<Plan> plans, xplans;
    std::vector<uint64_t> offs;
    BatchLayout lay;
    int st = plan_batch(p, count, prods, elem_bytes, plans, offs, &lay);
    if (st != PM_OK) return (pm_status)st;
    std::vector<pm_product> xprods;
    std::vector<UnwrapJob> jobs;
    expand_wrapped(plans, prods, elem_bytes, &xplans, &xprods, &jobs);
    layout_batch(xplans, offs, &lay);
    *out = lay.total;
    return PM_OK;
  } catch (const std::bad_alloc&) {
    return PM_ENOMEM;
  }
}

static pm_status batched_impl(uint64_t p, int32_t count, const pm_product* prods,
                              int elem_bytes, void* ws, uint64_t ws_bytes, void* stream);

// Host allocation failures of the batch bookkeeping become PM_ENOMEM.
static pm_status batched_common(uint64_t p, int32_t count, const pm_product* prods,
                                int elem_bytes, void* ws, uint64_t ws_bytes, void* stream) {
  return (pm_status)guarded(
      [&] { return (int)batched_impl(p, count, prods, elem_bytes, ws, ws_bytes, stream); });
}

static pm_status batched_impl(uint64_t p, int32_t count, const pm_product* prods,
                              int elem_bytes, void* ws, uint64_t ws_bytes, void* stream) {
  if (count < 0 || (count > 0 && !prods)) return PM_EINVAL;
  if (count == 0) return PM_OK;
  std::vector<Plan> plans, xplans;
  std::vector<uint64_t> offs;
  BatchLayout lay;
  int st = plan_batch(p, count, prods, elem_bytes, plans, offs, &lay);
  if (st != PM_OK) return (pm_status)st;
  std::vector<pm_product> xprods;
  std::vector<UnwrapJob> jobs;
  expand_wrapped(plans, prods, elem_bytes, &xplans, &xprods, &jobs);
  layout_batch(xplans, offs, &lay);
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < lay.total) return PM_EWORKSPACE;
  for (int32_t i = 0; i < count; ++i) {
    st = check_operands(plans[i], prods[i].A, prods[i].B, prods[i].C);
    if (st != PM_OK) return (pm_status)st;
    if (((uintptr_t)prods[i].A_eval | (uintptr_t)prods[i].B_eval) & 255) return PM_EINVAL;
    const uint64_t eb = (uint64_t)elem_bytes;
    const Plan& P = plans[i];
    st = check_workspace(ws, ws_bytes, lay.total, prods[i].A, eb * P.da * P.m * P.n, prods[i].B,
                         eb * P.db * P.n * P.k, prods[i].C, eb * (uint64_t)P.nout * P.m * P.k);
    if (st != PM_OK) return (pm_status)st;
  }
  const hipStream_t s = (hipStream_t)stream;
  st = run_batch(p, elem_bytes, xplans, offs, lay, xprods.data(), (uint8_t*)ws, ws_bytes, s);
  if (st != PM_OK) return (pm_status)st;
  for (const UnwrapJob& u : jobs) {
    KernelTimer kt(K_CRT, s);
    if (launch_unwrap(u.C, u.count, u.off, u.p, u.elem_bytes, s) != hipSuccess)
      return PM_EDEVICE;
  }
  return PM_OK;
}

static pm_status window_batched_impl(uint64_t p, int32_t count,
                                     const pm_window_product* wins, int elem_bytes, void* ws,
                                     uint64_t ws_bytes, void* stream);

static pm_status window_batched_common(uint64_t p, int32_t count,
                                       const pm_window_product* wins, int elem_bytes, void* ws,
                                       uint64_t ws_bytes, void* stream) {
  return (pm_status)guarded(
      [&] { return (int)window_batched_impl(p, count, wins, elem_bytes, ws, ws_bytes, stream); });
}

static pm_status window_batched_impl(uint64_t p, int32_t count,
                                     const pm_window_product* wins, int elem_bytes, void* ws,
                                     uint64_t ws_bytes, void* stream) {
  if (count < 0 || (count > 0 && !wins)) return PM_EINVAL;
  if (count == 0) return PM_OK;
  std::vector<Plan> plans;
  std::vector<uint64_t> offs;
  std::vector<pm_product> prods;
  BatchLayout lay;
  int st = plan_window_batch(p, count, wins, elem_bytes, plans, offs, &lay, &prods);
  if (st != PM_OK) return (pm_status)st;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < lay.total) return PM_EWORKSPACE;
  const uint64_t eb = (uint64_t)elem_bytes;
  for (int32_t i = 0; i < count; ++i) {
    const Plan& P = plans[i];
    st = check_operands(P, prods[i].A, prods[i].B, prods[i].C);
    if (st != PM_OK) return (pm_status)st;
    st = check_workspace(ws, ws_bytes, lay.total, prods[i].A, eb * P.da * P.m * P.n, prods[i].B,
                         eb * P.db * P.n * P.k, prods[i].C, eb * (uint64_t)P.nout * P.m * P.k);
    if (st != PM_OK) return (pm_status)st;
  }
  return (pm_status)run_batch(p, elem_bytes, plans, offs, lay, prods.data(), (uint8_t*)ws,
                              ws_bytes, (hipStream_t)stream);
}

pm_status pm_middle_batched_workspace_bytes(uint64_t p, int32_t count,
                                            const pm_window_product* wins, int32_t elem_bytes,
                                            uint64_t* out) {
  if (!out || count < 0 || (count > 0 && !wins)) return PM_EINVAL;
  try {
    std::vector<Plan> plans;
    std::vector<uint64_t> offs;
    BatchLayout lay;
    int st = plan_window_batch(p, count, wins, elem_bytes, plans, offs, &lay, nullptr);
    if (st != PM_OK) return (pm_status)st;
    *out = count ? lay.total : 0;
    return PM_OK;
  } catch (const std::bad_alloc&) {
    return PM_ENOMEM;
  }
}

pm_status pm_middle_batched_u32(uint32_t p, int32_t count, const pm_window_product* wins,
                                void* workspace, uint64_t workspace_bytes, void* stream) {
  return window_batched_common(p, count, wins, 4, workspace, workspace_bytes, stream);
}

pm_status pm_middle_batched_u64(uint64_t p, int32_t count, const pm_window_product* wins,
                                void* workspace, uint64_t workspace_bytes, void* stream) {
  return window_batched_common(p, count, wins, 8, workspace, workspace_bytes, stream);
}

pm_status pm_mul_batched_u32(uint32_t p, int32_t count, const pm_product* prods, void* workspace,
                             uint64_t workspace_bytes, void* stream) {
  return batched_common(p, count, prods, 4, workspace, workspace_bytes, stream);
}

pm_status pm_mul_batched_u64(uint64_t p, int32_t count, const pm_product* prods, void* workspace,
                             uint64_t workspace_bytes, void* stream) {
  return batched_common(p, count, prods, 8, workspace, workspace_bytes, stream);
}

}  // extern "C"
