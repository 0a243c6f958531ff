// pm_plan.cpp -- host planning: choice of transform prime(s), transform
// length, pass structure, tables of roots of unity, workspace layout.
//
// Method (Hyun, Neiger, Schost, ISSAC 2019, Section 2, "Polynomial matrix
// multiplication"): for FFT primes, evaluate and interpolate at roots of
// unity; for other moduli, lift the product to Z[x] and compute it modulo a
// few FFT primes ("3-primes" multiplication, Section 2, "Polynomial
// multiplication").  The product of two entries of degree < d has 2d-1
// coefficients, so L = 2^ceil(log2(2d-1)) points determine it.
#include "pm_plan.h"

#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <vector>

#include "../../include/pm.h"

namespace pm {

typedef unsigned __int128 u128;

namespace {
std::atomic<int> g_fail_countdown{-1};
}

void alloc_point() {
  if (g_fail_countdown.load(std::memory_order_relaxed) < 0) return;
  if (g_fail_countdown.fetch_sub(1) == 0) throw std::bad_alloc();
}

uint64_t powmod_u64(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = (uint64_t)((u128)r * b % m);
    b = (uint64_t)((u128)b * b % m);
    e >>= 1;
  }
  return r;
}

int v2_u64(uint64_t x) {
  if (x == 0) return 64;
  int v = 0;
  while ((x & 1) == 0) { x >>= 1; ++v; }
  return v;
}

// Deterministic Miller-Rabin for 64-bit n (bases: the primes up to 37).
static bool miller_rabin_u64(uint64_t n) {
  static const uint64_t B[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t b : B)
    if (n % b == 0) return n == b;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t b : B) {
    uint64_t x = powmod_u64(b, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s && comp; ++i) {
      x = (uint64_t)((u128)x * x % n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

// The planner asks about the same few moduli on every call, and the test
// costs a few microseconds: the last answers are kept per thread.
bool is_prime_u64(uint64_t n) {
  thread_local uint64_t seen[4] = {0, 0, 0, 0};
  thread_local bool answer[4] = {false, false, false, false};
  thread_local int next = 0;
  for (int i = 0; i < 4; ++i)
    if (seen[i] == n && n != 0) return answer[i];
  const bool r = miller_rabin_u64(n);
  seen[next] = n;
  answer[next] = r;
  next = (next + 1) & 3;
  return r;
}

// Primes q < 2^31 with 2^24 | q-1, largest first.  Each supports transforms
// up to length 2^24, above the 2^15 this library runs in LDS.
static const uint32_t kCrtPrimes[] = {
    2130706433u,  // 127 * 2^24 + 1
    2113929217u,  //  63 * 2^25 + 1
    2013265921u,  //  15 * 2^27 + 1
    1811939329u,  //  27 * 2^26 + 1
    1711276033u,  //  51 * 2^25 + 1
    1224736769u,  //  73 * 2^24 + 1
    1107296257u,  //  33 * 2^25 + 1
    754974721u,   //  45 * 2^24 + 1
    469762049u,   //   7 * 2^26 + 1
    167772161u,   //   5 * 2^25 + 1
};

// Primes q with 2q - 1 <= 0x7F7F7F7F (below 2^30) and 2^20 | q-1, largest
// first: their transforms run lazy butterflies (residues kept in [0, 2q)).
static const uint32_t kCrtPrimesLazy[] = {
    1053818881u,  // 1005 * 2^20 + 1
    1051721729u,  // 1003 * 2^20 + 1
    1045430273u,  //  997 * 2^20 + 1
    1012924417u,  //  483 * 2^21 + 1
    1007681537u,  //  961 * 2^20 + 1
    1004535809u,  //  479 * 2^21 + 1
    998244353u,   //  119 * 2^23 + 1
    985661441u,   //  235 * 2^22 + 1
};

// split: stages of the column pass (0: none; kept below logL by the
// planner); maxr: most stages per later pass.
PassPlan make_pass_plan(int logL, int split, int maxr) {
  PassPlan P{};
  P.logL = logL;
  P.split = split;
  int rest = logL, first = 0;
  if (P.split) {
    P.stages[0] = P.split;
    rest -= P.split;
    first = 1;
  }
  if (maxr < 2) maxr = 2;
  // at most maxr stages per pass, and at most kMaxPasses passes
  while (maxr < 4 && first + (rest + maxr - 1) / maxr > kMaxPasses) ++maxr;
  const int nrest = (rest + maxr - 1) / maxr;
  P.npass = first + nrest;
  for (int i = 0; i < nrest; ++i)
    P.stages[first + i] = rest / nrest + (i < rest % nrest ? 1 : 0);
  int s = logL;
  uint32_t off = 0;
  for (int i = 0; i < P.npass; ++i) {
    s -= P.stages[i];
    P.stride_log[i] = s;
    P.tw_off[i] = off;
    off += (1u << s) * ((1u << P.stages[i]) - 1);
  }
  P.tw_count = off;
  return P;
}

// Exact multi-precision helpers for the CRT bound (little-endian 32-bit limbs).
typedef std::vector<uint32_t> Big;
static Big big_from(uint64_t v) { return Big{(uint32_t)v, (uint32_t)(v >> 32)}; }
static Big big_mul(const Big& a, uint64_t b) {
  Big r(a.size() + 2, 0);
  uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  for (int part = 0; part < 2; ++part) {
    uint64_t bb = part ? b1 : b0, carry = 0;
    for (size_t i = 0; i < a.size(); ++i) {
      u128 t = (u128)a[i] * bb + r[i + part] + carry;
      r[i + part] = (uint32_t)t;
      carry = (uint64_t)(t >> 32);
    }
    for (size_t i = a.size() + part; carry && i < r.size(); ++i) {
      uint64_t t = (uint64_t)r[i] + carry;
      r[i] = (uint32_t)t;
      carry = t >> 32;
    }
  }
  while (r.size() > 1 && r.back() == 0) r.pop_back();
  return r;
}
static int big_cmp(const Big& a, const Big& b) {
  size_t n = a.size() > b.size() ? a.size() : b.size();
  for (size_t i = n; i-- > 0;) {
    uint32_t x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}

static int ceil_log2(uint64_t x) {
  int l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

// Pointwise variant: int8-MFMA limbs where the shape allows (contraction
// length a multiple of 4 and below 2^12, both matrices' limb planes within
// the 160 KiB of LDS of a CU) and `want` is 1, else the VALU kernel.
int choose_pointwise(int m, int n, int k, int want) {
  const uint64_t mp = (m + 15) & ~15, kp = (k + 15) & ~15, np = (n + 63) & ~63;
  const bool mfma_ok = n % 4 == 0 && n < 4096 && 4 * (mp + kp) * (np + 16) <= 160 * 1024;
  return want && mfma_ok ? 1 : 0;
}

static int make_plan_core(uint64_t p, int m, int n, int k, int da, int db, int lo, int nout,
                          int elem_bytes, int force_log, Plan* out);

int make_slice_plan(uint64_t p, int m, int n, int k, int da, int db, int lo, int nout,
                    int elem_bytes, Plan* out) {
  return make_plan_core(p, m, n, k, da, db, lo, nout, elem_bytes, -1, out);
}

int make_cyclic_plan(uint64_t p, int m, int n, int k, int d, int logL, int elem_bytes,
                     Plan* out) {
  if (logL < 0 || logL > kMaxLogLen || d < 1 || d > (1 << logL)) return PM_EINVAL;
  return make_plan_core(p, m, n, k, d, d, 0, std::min(1 << logL, 2 * d - 1), elem_bytes, logL,
                        out);
}

static int make_plan_core(uint64_t p, int m, int n, int k, int da, int db, int lo, int nout,
                          int elem_bytes, int force_log, Plan* out) {
  if (!out) return PM_EINVAL;
  alloc_point();  // the CRT bound below uses heap big integers
  if (elem_bytes != 4 && elem_bytes != 8) return PM_EINVAL;
  if (m < 1 || n < 1 || k < 1 || da < 1 || db < 1 || lo < 0 || nout < 1) return PM_EINVAL;
  if (p < 2) return PM_EINVAL;
  // the window must lie inside the product's da + db - 1 coefficients
  if ((uint64_t)lo + (uint64_t)nout > (uint64_t)da + (uint64_t)db - 1) return PM_EINVAL;
  if (elem_bytes == 4 && p > 0xFFFFFFFFull) return PM_ERANGE;
  if (elem_bytes == 8 && p >= (1ull << 62)) return PM_ERANGE;
  const uint64_t need = std::max<uint64_t>((uint64_t)da + db - 1 - lo, (uint64_t)lo + nout);
  // a forced length computes A B mod (x^L - 1) (coefficients wrap)
  const int logL = force_log >= 0 ? force_log : ceil_log2(need);
  if (logL > kMaxLogLen) return PM_EUNSUPPORTED;
  const uint64_t L = 1ull << logL;
  const uint64_t lim = 1ull << 32;
  const uint64_t mn = (uint64_t)m * n, nk = (uint64_t)n * k, mk = (uint64_t)m * k;
  if ((uint64_t)da * mn >= lim || (uint64_t)db * nk >= lim || (uint64_t)nout * mk >= lim ||
      L * mn >= lim || L * nk >= lim || L * mk >= lim)
    return PM_ERANGE;

  Plan P{};
  P.p = p; P.m = m; P.n = n; P.k = k; P.elem_bytes = elem_bytes;
  P.d = std::max(da, db);
  P.da = da; P.db = db; P.lo = lo; P.nout = nout;
  P.logL = logL;
  if (p >= 3 && p < (1ull << 31) && is_prime_u64(p) && v2_u64(p - 1) >= logL) {
    P.mode = 0;
    P.r = 1;
    P.q[0] = (uint32_t)p;
  } else {
    // Integer coefficients of the lifted product lie in
    // [0, n * min(da, db) * (p-1)^2]; so do those of a cyclic product with
    // da = db = d <= L, since a + b = c mod L has at most one solution b in
    // [0, d) for each a.
    Big bound = big_mul(big_mul(big_from(p - 1), p - 1), (uint64_t)n * std::min(da, db));
    Big prod = big_from(1);
    P.mode = 1;
    P.r = 0;
    for (uint32_t q : kCrtPrimes) {
      if (v2_u64(q - 1) < logL) continue;
      if (P.r == kMaxPrimes) return PM_EUNSUPPORTED;
      P.q[P.r++] = q;
      prod = big_mul(prod, q);
      if (big_cmp(prod, bound) > 0) break;
    }
    if (big_cmp(prod, bound) <= 0) return PM_EUNSUPPORTED;
    // As many primes below 2^30 suffice for most products: take those, whose
    // transforms keep lazy residues.
    Big lprod = big_from(1);
    uint32_t lq[kMaxPrimes];
    int lr = 0;
    for (uint32_t q : kCrtPrimesLazy) {
      if (lr == P.r) break;
      if (v2_u64(q - 1) < logL) continue;
      lq[lr++] = q;
      lprod = big_mul(lprod, q);
    }
    if (lr == P.r && big_cmp(lprod, bound) > 0)
      for (int i = 0; i < lr; ++i) P.q[i] = lq[i];
  }
  const int pclass = P.mode == 1 ? kClassCrt : P.q[0] < (1u << 30) ? kClassDirectLt30
                                                                     : kClassDirectGe30;
  P.kn = tuned_knobs(pclass, logL, m, n, k, &P.tune_entry);
  const GlobalKnobs& G = global_knobs();
  if (P.kn.split < 2 || logL < G.split_min_log || P.kn.split >= logL) P.kn.split = 0;
  P.pointwise = choose_pointwise(m, n, k, P.kn.pointwise);
  // Three-quarter transforms (split transforms of whole products whose
  // da + db - 1 coefficients fit in 3L/4 points; global knob trunc34).
  P.trunc = 0;
  P.npts = (int)L;
  P.keep = P.kn.split ? 1 << P.kn.split : 1;
  if (G.trunc34 && force_log < 0 && lo == 0 && (uint64_t)nout == (uint64_t)da + db - 1 &&
      P.kn.split >= 2 && 4 * need <= 3 * L) {
    P.trunc = 1;
    P.npts = (int)(3 * L / 4);
    P.keep = 3 << (P.kn.split - 2);
  }
  const uint64_t np = (uint64_t)P.npts;
  uint64_t off = 0;
  P.off_ahat = off; off = align_up(off + 4 * np * mn, 256);
  P.off_bhat = off; off = align_up(off + 4 * np * nk, 256);
  P.off_chat = off; off = align_up(off + 4 * np * mk, 256);
  P.prime_stride = off;
  P.off_cq = P.prime_stride * (uint64_t)P.r;
  P.ws_bytes = P.off_cq;
  if (P.mode == 1) P.ws_bytes = align_up(P.off_cq + 4ull * P.r * (uint64_t)nout * mk, 256);
  *out = P;
  return PM_OK;
}

int make_plan(uint64_t p, int m, int n, int k, int d, int elem_bytes, Plan* out) {
  if (d < 1) return PM_EINVAL;
  return make_slice_plan(p, m, n, k, d, d, 0, 2 * d - 1, elem_bytes, out);
}

}  // namespace pm

extern "C" pm_status pm_debug_fail_alloc(int32_t countdown) {
  pm::g_fail_countdown.store(countdown < 0 ? -1 : countdown);
  return PM_OK;
}
