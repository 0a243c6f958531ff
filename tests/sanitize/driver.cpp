// Host-code driver for the AddressSanitizer / UndefinedBehaviorSanitizer
// build (tests/test_sanitizers_cpu.py): exercises every path of the C ABI
// that runs before device work (planning, size queries, argument checks,
// the tuning-table parser, the host M-Basis and matrix inverse, injected
// allocation failures), and the oracle's functions, on a machine without a
// GPU.  Exits non-zero on a wrong status; the sanitizers abort on a memory
// or undefined-behaviour error.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "pm.h"

extern "C" {
int orc_polymatmul(uint64_t p, int m, int n, int k, int d, const uint64_t* A,
                   const uint64_t* B, uint64_t* C, int threads);
int orc_polymatmul_entries(uint64_t p, int m, int n, int k, int d, const uint64_t* A,
                           const uint64_t* B, int count, const int32_t* ii, const int32_t* jj,
                           uint64_t* out, int threads);
void orc_eval_points(uint64_t p, int rows, int cols, int deg, const uint64_t* X, int npts,
                     const uint64_t* pts, uint64_t* out, int threads);
void orc_project_left_mt(uint64_t p, int rows, int cols, int deg, const uint64_t* X,
                         const uint64_t* u, uint64_t* out, int threads);
void orc_project_right_mt(uint64_t p, int rows, int cols, int deg, const uint64_t* X,
                          const uint64_t* v, uint64_t* out, int threads);
void orc_polymul_sum(uint64_t p, int n, int d, const uint64_t* U, const uint64_t* V,
                     uint64_t* out, int threads);
int orc_is_prime(uint64_t n);
}

static int failures = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);   \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

static std::mt19937_64 rng(20190507);

static std::vector<uint64_t> residues(size_t n, uint64_t p) {
  std::vector<uint64_t> v(n);
  for (auto& x : v) x = rng() % p;
  return v;
}

static void plans() {
  const uint64_t ps[] = {2, 3, 97, 998244353, 2013265921, 4294967291ull, 1ull << 31,
                         (1ull << 61) - 1, (1ull << 62) - 57, 1ull << 40, 1000000007};
  const int dims[] = {1, 2, 3, 7, 16, 33, 128, 4096};
  const int degs[] = {1, 2, 3, 100, 1025, 4096, 4097, 16384, 16385, 1 << 20};
  pm_plan_info info;
  uint64_t out = 0;
  for (uint64_t p : ps)
    for (int eb : {4, 8})
      for (int m : dims)
        for (int d : degs) {
          const int st = pm_plan(p, m, 3, (m % 5) + 1, d, eb, &info);
          CHECK(st == PM_OK || st == PM_ERANGE || st == PM_EUNSUPPORTED || st == PM_EINVAL);
          if (st == PM_OK) {
            CHECK(info.num_primes >= 1 && info.num_primes <= 8);
            CHECK(pm_workspace_bytes(p, m, 3, (m % 5) + 1, d, eb, &out) == PM_OK);
            CHECK(out == info.workspace_bytes);
            CHECK(pm_tables_bytes(p, m, 3, (m % 5) + 1, d, eb, &out) == PM_OK);
          }
        }
  // sizes whose products overflow 32 bits, and bad arguments
  CHECK(pm_plan(97, 1 << 16, 1 << 16, 1, 2, 4, &info) == PM_ERANGE);
  CHECK(pm_plan(97, 0, 1, 1, 1, 4, &info) == PM_EINVAL);
  CHECK(pm_plan(97, 1, 1, 1, 1, 3, &info) == PM_EINVAL);
  CHECK(pm_plan(97, 1, 1, 1, 1, 4, nullptr) == PM_EINVAL);
  CHECK(pm_plan(1, 1, 1, 1, 1, 4, &info) == PM_EINVAL);
  // windows
  for (int lo = 0; lo < 40; lo += 7)
    for (int len = 1; len < 40; len += 9) {
      const int st = pm_middle_plan(998244353, 2, 3, 2, 20, 21, lo, len, 4, &info);
      CHECK(st == (lo + len <= 40 ? PM_OK : PM_EINVAL));
    }
}

static void argument_checks() {
  const uintptr_t A = 1 << 20, B = 2 << 20, C = 3 << 20, W = 64 << 20;
  uint64_t need = 0;
  CHECK(pm_workspace_bytes(998244353, 4, 4, 4, 16, 4, &need) == PM_OK);
  // NULL, misaligned, overlapping, too small: all rejected before device work
  CHECK(pm_mul_u32(998244353, 4, 4, 4, 16, nullptr, (uint32_t*)B, (uint32_t*)C, (void*)W,
                   need, nullptr) == PM_EINVAL);
  CHECK(pm_mul_u32(998244353, 4, 4, 4, 16, (uint32_t*)(A + 4), (uint32_t*)B, (uint32_t*)C,
                   (void*)W, need, nullptr) == PM_EINVAL);
  CHECK(pm_mul_u32(998244353, 4, 4, 4, 16, (uint32_t*)A, (uint32_t*)B, (uint32_t*)A,
                   (void*)W, need, nullptr) == PM_EINVAL);
  CHECK(pm_mul_u32(998244353, 4, 4, 4, 16, (uint32_t*)A, (uint32_t*)B, (uint32_t*)C,
                   (void*)W, need - 1, nullptr) == PM_EWORKSPACE);
  CHECK(pm_mul_u64((1ull << 62), 4, 4, 4, 16, (uint64_t*)A, (uint64_t*)B, (uint64_t*)C,
                   (void*)W, need, nullptr) == PM_ERANGE);
  CHECK(pm_mul_noalloc(2013265921, 64, 64, 32, 4096, 4, (void*)A, (void*)B, (void*)C,
                       nullptr) == PM_ESCRATCH);
  // batches: sizes, then a bad product anywhere in the array
  std::vector<pm_product> prods(37);
  for (size_t i = 0; i < prods.size(); ++i) {
    pm_product& q = prods[i];
    memset(&q, 0, sizeof q);
    q.m = 1 + (int)(rng() % 9);
    q.n = 1 + (int)(rng() % 9);
    q.k = 1 + (int)(rng() % 9);
    q.d = 1 + (int)(rng() % 3000);
    q.A = (void*)(A + (i << 12));
    q.B = (void*)(B + (i << 12));
    q.C = (void*)(C + (i << 16));
  }
  CHECK(pm_batched_workspace_bytes(998244353, (int)prods.size(), prods.data(), 4, &need) ==
        PM_OK);
  prods[17].d = 0;
  CHECK(pm_batched_workspace_bytes(998244353, (int)prods.size(), prods.data(), 4, &need) ==
        PM_EINVAL);
  CHECK(pm_mul_batched_u32(998244353, (int)prods.size(), prods.data(), (void*)W, 1ull << 40,
                           nullptr) == PM_EINVAL);
  std::vector<pm_window_product> wins(5);
  for (size_t i = 0; i < wins.size(); ++i) {
    memset(&wins[i], 0, sizeof wins[i]);
    wins[i].m = 2; wins[i].n = 3; wins[i].k = 2; wins[i].da = 10; wins[i].db = 19;
    wins[i].lo = 9; wins[i].len = 10;
    wins[i].A = (void*)(A + (i << 12));
    wins[i].B = (void*)(B + (i << 12));
    wins[i].C = (void*)(C + (i << 16));
  }
  CHECK(pm_middle_batched_workspace_bytes(998244353, 5, wins.data(), 4, &need) == PM_OK);
  wins[3].lo = 100;
  CHECK(pm_middle_batched_workspace_bytes(998244353, 5, wins.data(), 4, &need) == PM_EINVAL);
  CHECK(pm_tables_attach(nullptr, 1 << 20) == PM_EINVAL);
  CHECK(pm_neg_mod(97, (void*)A, (void*)(A + 4), 4, 4, nullptr) == PM_EINVAL);
  for (int s = -9; s <= 0; ++s) CHECK(pm_status_str(s) != nullptr);
}

static void tuning_tables() {
  CHECK(pm_tune_load("") == PM_OK);
  const char* good =
      "{\"format\": \"pm-tune-1\", \"global\": {\"wrap_min_log\": 11, \"min_wg\": 64},"
      " \"entries\": [{\"prime_class\": \"direct_ge30\", \"log2_len\": 13, \"m_log2\": 6,"
      " \"knobs\": {\"split\": 3, \"maxr\": 2, \"blk_nt\": 512}, \"us\": 1.5e2},"
      " {\"knobs\": {\"pointwise\": 0}}]}";
  CHECK(pm_tune_load(good) == PM_OK);
  pm_plan_info info;
  CHECK(pm_plan(2013265921, 64, 64, 32, 4096, 4, &info) == PM_OK && info.tune_entry == 0);
  CHECK(pm_plan(998244353, 8, 8, 8, 256, 4, &info) == PM_OK && info.tune_entry == 1);
  // every truncation and single-byte change of a valid table: accepted or
  // rejected, never a crash
  const std::string g = good;
  for (size_t cut = 0; cut < g.size(); ++cut) {
    const std::string t = g.substr(0, cut);
    const int st = pm_tune_load(t.c_str());
    CHECK(st == PM_OK || st == PM_EINVAL);
  }
  const char alphabet[] = "{}[]\":,0123456789-+.eE \\nulltruefalsexyz";
  for (int it = 0; it < 4000; ++it) {
    std::string t = g;
    const int edits = 1 + (int)(rng() % 3);
    for (int e = 0; e < edits; ++e)
      t[rng() % t.size()] = alphabet[rng() % (sizeof alphabet - 1)];
    const int st = pm_tune_load(t.c_str());
    CHECK(st == PM_OK || st == PM_EINVAL);
  }
  std::string deep(5000, '[');
  CHECK(pm_tune_load(deep.c_str()) == PM_EINVAL);
  CHECK(pm_tune_load("") == PM_OK);
}

static void host_algorithms() {
  const uint64_t ps[] = {2, 97, 998244353, (1ull << 61) - 1, (1ull << 62) - 57};
  for (uint64_t p : ps)
    for (int m : {1, 3, 6, 20})
      for (int n : {1, 2, 4, 16}) {
        if (m == 20 && p < 97) continue;
        const int sigma = m == 20 ? 3 : 7;
        std::vector<uint64_t> F = residues((size_t)sigma * m * n, p);
        std::vector<int64_t> shift(m);
        for (auto& s : shift) s = (int64_t)(rng() % 7) - 3;
        std::vector<uint64_t> P((size_t)(sigma + 1) * m * m);
        std::vector<int64_t> rd(m);
        CHECK(pm_mbasis_host(p, m, n, sigma, F.data(), shift.data(), P.data(), rd.data()) ==
              PM_OK);
      }
  CHECK(pm_mbasis_host(100, 2, 1, 3, nullptr, nullptr, nullptr, nullptr) == PM_EINVAL);
  for (uint64_t p : {97ull, 998244353ull, (1ull << 62) - 57})
    for (int n : {1, 2, 5, 17}) {
      std::vector<uint64_t> M = residues((size_t)n * n, p), Mi((size_t)n * n);
      const int st = pm_matinv_host(p, n, M.data(), Mi.data());
      CHECK(st == PM_OK || st == PM_EINVAL);
    }
}

static void injected_failures() {
  std::vector<pm_product> prods(3);
  for (size_t i = 0; i < prods.size(); ++i) {
    memset(&prods[i], 0, sizeof prods[i]);
    prods[i].m = 4; prods[i].n = 4; prods[i].k = 4; prods[i].d = 100 * (int)(i + 1);
    prods[i].A = (void*)(uintptr_t)((1 + i) << 20);
    prods[i].B = (void*)(uintptr_t)((8 + i) << 20);
    prods[i].C = (void*)(uintptr_t)((16 + i) << 20);
  }
  std::vector<uint64_t> F = residues(5 * 4 * 2, 97), P(6 * 4 * 4);
  std::vector<int64_t> shift(4, 0), rd(4);
  for (int countdown = 0; countdown < 12; ++countdown) {
    uint64_t need = 0;
    pm_plan_info info;
    CHECK(pm_debug_fail_alloc(countdown) == PM_OK);
    int st = pm_batched_workspace_bytes(998244353, 3, prods.data(), 4, &need);
    CHECK(st == PM_OK || st == PM_ENOMEM);
    CHECK(pm_debug_fail_alloc(countdown) == PM_OK);
    st = pm_mbasis_host(97, 4, 2, 5, F.data(), shift.data(), P.data(), rd.data());
    CHECK(st == PM_OK || st == PM_ENOMEM);
    CHECK(pm_debug_fail_alloc(countdown) == PM_OK);
    st = pm_plan((1ull << 61) - 1, 8, 8, 8, 1000, 8, &info);
    CHECK(st == PM_OK || st == PM_ENOMEM);
    CHECK(pm_debug_fail_alloc(countdown) == PM_OK);
    st = pm_tune_load("{\"format\": \"pm-tune-1\", \"entries\": [{\"knobs\": {\"maxr\": 3}}]}");
    CHECK(st == PM_OK || st == PM_ENOMEM);
  }
  CHECK(pm_debug_fail_alloc(-1) == PM_OK);
  CHECK(pm_tune_load("") == PM_OK);
}

static void oracle() {
  for (uint64_t p : {2ull, 97ull, 2013265921ull, (1ull << 62) - 57}) {
    const int m = 3, n = 4, k = 2, d = 9;
    std::vector<uint64_t> A = residues((size_t)d * m * n, p), B = residues((size_t)d * n * k, p);
    std::vector<uint64_t> C((size_t)(2 * d - 1) * m * k);
    CHECK(orc_polymatmul(p, m, n, k, d, A.data(), B.data(), C.data(), 3) == 0);
    const int32_t ii[2] = {0, 2}, jj[2] = {1, 0};
    std::vector<uint64_t> E(2 * (2 * d - 1));
    CHECK(orc_polymatmul_entries(p, m, n, k, d, A.data(), B.data(), 2, ii, jj, E.data(), 2) ==
          0);
    CHECK(E[0] == C[1] && E[2 * d - 1] == C[2 * k]);
    const uint64_t pts[3] = {0, 1, p - 1};
    std::vector<uint64_t> ev(3 * m * n);
    orc_eval_points(p, m, n, d, A.data(), 3, pts, ev.data(), 4);
    std::vector<uint64_t> u = residues(m, p), v = residues(k, p), uA((size_t)d * n),
                          Bv((size_t)d * n), s(2 * d - 1);
    orc_project_left_mt(p, m, n, d, A.data(), u.data(), uA.data(), 2);
    orc_project_right_mt(p, n, k, d, B.data(), v.data(), Bv.data(), 2);
    orc_polymul_sum(p, n, d, uA.data(), Bv.data(), s.data(), 3);
    CHECK(orc_is_prime(p) == 1);
  }
}

int main() {
  plans();
  argument_checks();
  tuning_tables();
  host_algorithms();
  injected_failures();
  oracle();
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("sanitized host driver: ok\n");
  return 0;
}
