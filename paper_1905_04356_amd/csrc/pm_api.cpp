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
#include <string.h>

#include <new>

#include "../../include/pm.h"
#include "pm_kernels.h"
#include "pm_plan.h"
#include "pm_profile.h"

using namespace pm;

extern "C" {

const char* pm_status_str(int status) {
  switch (status) {
    case PM_OK: return "PM_OK";
    case PM_EINVAL: return "PM_EINVAL: invalid argument";
    case PM_ERANGE: return "PM_ERANGE: modulus or size out of range";
    case PM_ENOMEM: return "PM_ENOMEM: table allocation failed";
    case PM_EWORKSPACE: return "PM_EWORKSPACE: workspace missing, misaligned or too small";
    case PM_EDEVICE: return "PM_EDEVICE: HIP error";
    case PM_EUNSUPPORTED: return "PM_EUNSUPPORTED: length or bound not supported";
    case PM_EBUSY: return "PM_EBUSY: busy";
    default: return "unknown pm_status";
  }
}

int pm_abi_version(void) { return PM_ABI_VERSION; }

pm_status pm_plan(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d, int32_t elem_bytes,
                  pm_plan_info* out) {
  if (!out) return PM_EINVAL;
  Plan P;
  int st = make_plan(p, m, n, k, d, elem_bytes, &P);
  if (st != PM_OK) return (pm_status)st;
  memset(out, 0, sizeof *out);
  out->mode = P.mode;
  out->log2_len = P.logL;
  out->num_primes = P.r;
  out->pointwise = P.pointwise;
  for (int i = 0; i < P.r; ++i) out->primes[i] = P.q[i];
  out->workspace_bytes = P.ws_bytes;
  return PM_OK;
}

pm_status pm_workspace_bytes(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d,
                             int32_t elem_bytes, uint64_t* out) {
  if (!out) return PM_EINVAL;
  Plan P;
  int st = make_plan(p, m, n, k, d, elem_bytes, &P);
  if (st != PM_OK) return (pm_status)st;
  *out = P.ws_bytes;
  return PM_OK;
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
  const uint64_t na = eb * P.d * P.m * P.n, nb = eb * P.d * P.n * P.k;
  const uint64_t nc = eb * (2ull * P.d - 1) * P.m * P.k;
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
  for (int i = 0; i < P.r; ++i) {
    const uint32_t qi = P.q[i];
    c->q[i] = qi;
    c->mu[i] = ~0ull / qi;
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

// Enqueue one product.  A, B, C are device pointers of elem_bytes residues.
int run_product(const Plan& P, const void* A, const void* B, void* C, uint8_t* ws,
                hipStream_t s) {
  PrimeConst pc[kMaxPrimes];
  for (int i = 0; i < P.r; ++i) {
    int st = get_prime_const(P.q[i], P.logL, &pc[i]);
    if (st != PM_OK) return st;
  }
  const int m = P.m, n = P.n, k = P.k, d = P.d;
  const uint64_t pstride = P.prime_stride / 4;  // in u32 elements
  uint32_t* ahat = (uint32_t*)(ws + P.off_ahat);
  uint32_t* bhat = (uint32_t*)(ws + P.off_bhat);
  uint32_t* chat = (uint32_t*)(ws + P.off_chat);
  // In direct mode the inputs are already residues mod q = p.
  const int reduce = P.mode == 1;

  NttLaunch fa;
  memset(&fa, 0, sizeof fa);
  fill_ntt_launch(&fa, P.logL, m * n, d);
  for (int i = 0; i < P.r; ++i) fa.pc[i] = pc[i];
  fa.in = A;
  fa.out = ahat;
  fa.in_prime_stride = 0;
  fa.out_prime_stride = pstride;
  {
    KernelTimer kt(K_NTT_FWD, s);
    if (launch_ntt_fwd(fa, P.elem_bytes, reduce, P.r, s) != hipSuccess) return PM_EDEVICE;
  }

  NttLaunch fb = fa;
  fill_ntt_launch(&fb, P.logL, n * k, d);
  fb.in = B;
  fb.out = bhat;
  {
    KernelTimer kt(K_NTT_FWD, s);
    if (launch_ntt_fwd(fb, P.elem_bytes, reduce, P.r, s) != hipSuccess) return PM_EDEVICE;
  }

  PointwiseLaunch pw;
  memset(&pw, 0, sizeof pw);
  pw.m = m; pw.n = n; pw.k = k; pw.L = 1 << P.logL;
  pw.prime_stride = pstride;
  pw.ahat = ahat; pw.bhat = bhat; pw.chat = chat;
  for (int i = 0; i < P.r; ++i) {
    pw.pc[i] = pc[i];
    // weights of the limb accumulators: 256^s L^{-1} mod q
    uint64_t w = pc[i].linv;
    for (int t = 0; t < 7; ++t) {
      pw.cs[i][t] = (uint32_t)w;
      w = (w << 8) % P.q[i];
    }
  }
  {
    KernelTimer kt(K_POINTWISE, s);
    const int st = P.pointwise == 1 ? launch_pointwise_mfma(pw, P.r, s)
                                    : launch_pointwise(pw, P.r, s);
    if (st != hipSuccess) return PM_EDEVICE;
  }

  NttLaunch ic = fa;
  fill_ntt_launch(&ic, P.logL, m * k, 2 * d - 1);
  ic.in = chat;
  ic.in_prime_stride = pstride;
  if (P.mode == 0) {
    ic.out = C;
    ic.out_prime_stride = 0;
    KernelTimer kt(K_NTT_INV, s);
    if (launch_ntt_inv(ic, P.elem_bytes, 1, s) != hipSuccess) return PM_EDEVICE;
    return PM_OK;
  }
  uint32_t* cq = (uint32_t*)(ws + P.off_cq);
  const uint64_t nout = (2ull * d - 1) * m * k;
  ic.out = cq;
  ic.out_prime_stride = nout;
  {
    KernelTimer kt(K_NTT_INV, s);
    if (launch_ntt_inv(ic, 4, P.r, s) != hipSuccess) return PM_EDEVICE;
  }
  CrtLaunch cr;
  fill_crt(P, &cr);
  cr.count = nout;
  cr.prime_stride = nout;
  cr.cq = cq;
  cr.out = C;
  KernelTimer kt(K_CRT, s);
  if (launch_crt(cr, P.elem_bytes, s) != hipSuccess) return PM_EDEVICE;
  return PM_OK;
}

pm_status mul_common(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d, int elem_bytes,
                     const void* A, const void* B, void* C, void* ws, uint64_t ws_bytes,
                     void* stream) {
  Plan P;
  int st = make_plan(p, m, n, k, d, elem_bytes, &P);
  if (st != PM_OK) return (pm_status)st;
  st = check_operands(P, A, B, C);
  if (st != PM_OK) return (pm_status)st;
  const uint64_t eb = (uint64_t)elem_bytes;
  st = check_workspace(ws, ws_bytes, P.ws_bytes, A, eb * d * m * n, B, eb * d * n * k, C,
                       eb * (2ull * d - 1) * m * k);
  if (st != PM_OK) return (pm_status)st;
  return (pm_status)run_product(P, A, B, C, (uint8_t*)ws, (hipStream_t)stream);
}

}  // namespace

extern "C" {

pm_status pm_mul_u32(uint32_t p, int32_t m, int32_t n, int32_t k, int32_t d, const uint32_t* A,
                     const uint32_t* B, uint32_t* C, void* workspace, uint64_t workspace_bytes,
                     void* stream) {
  return mul_common(p, m, n, k, d, 4, A, B, C, workspace, workspace_bytes, stream);
}

pm_status pm_mul_u64(uint64_t p, int32_t m, int32_t n, int32_t k, int32_t d, const uint64_t* A,
                     const uint64_t* B, uint64_t* C, void* workspace, uint64_t workspace_bytes,
                     void* stream) {
  return mul_common(p, m, n, k, d, 8, A, B, C, workspace, workspace_bytes, stream);
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

// ---- batched products ---------------------------------------------------------

namespace {

int plan_batch(uint64_t p, int32_t count, const pm_product* prods, int32_t elem_bytes,
               Plan* plans, uint64_t* total) {
  uint64_t off = 0;
  for (int32_t i = 0; i < count; ++i) {
    const pm_product& pr = prods[i];
    int st = make_plan(p, pr.m, pr.n, pr.k, pr.d, elem_bytes, &plans[i]);
    if (st != PM_OK) return st;
    off = align_up(off + plans[i].ws_bytes, 256);
  }
  *total = off;
  return PM_OK;
}

}  // namespace

extern "C" {

pm_status pm_batched_workspace_bytes(uint64_t p, int32_t count, const pm_product* prods,
                                     int32_t elem_bytes, uint64_t* out) {
  if (!out || count < 0 || (count > 0 && !prods)) return PM_EINVAL;
  Plan* plans = new (std::nothrow) Plan[count > 0 ? count : 1];
  if (!plans) return PM_ENOMEM;
  uint64_t total = 0;
  int st = plan_batch(p, count, prods, elem_bytes, plans, &total);
  delete[] plans;
  if (st != PM_OK) return (pm_status)st;
  *out = total;
  return PM_OK;
}

static pm_status batched_common(uint64_t p, int32_t count, const pm_product* prods,
                                int elem_bytes, void* ws, uint64_t ws_bytes, void* stream) {
  if (count < 0 || (count > 0 && !prods)) return PM_EINVAL;
  if (count == 0) return PM_OK;
  Plan* plans = new (std::nothrow) Plan[count];
  if (!plans) return PM_ENOMEM;
  uint64_t total = 0;
  int st = plan_batch(p, count, prods, elem_bytes, plans, &total);
  for (int32_t i = 0; st == PM_OK && i < count; ++i)
    st = check_operands(plans[i], prods[i].A, prods[i].B, prods[i].C);
  if (st == PM_OK && (!ws || ((uintptr_t)ws & 255) || ws_bytes < total)) st = PM_EWORKSPACE;
  uint64_t off = 0;
  for (int32_t i = 0; st == PM_OK && i < count; ++i) {
    st = run_product(plans[i], prods[i].A, prods[i].B, prods[i].C, (uint8_t*)ws + off,
                     (hipStream_t)stream);
    off = align_up(off + plans[i].ws_bytes, 256);
  }
  delete[] plans;
  return (pm_status)st;
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
