// pm_mbasis.cpp -- Algorithm M-Basis on the host: the leaves of PM-Basis.
//
// Hyun, Neiger, Schost (ISSAC 2019), Section 3, "Approximant bases": for F in
// K[x]^{m x n} and order sigma, M-Basis runs sigma rounds; round k takes the
// residual R (coefficient k of P F), the s'-Popov approximant basis Q of R at
// order 1 (M-Basis-1), and sets P := Q P, s' := rdeg_s(P).
//
// M-Basis-1 on a constant R: rows are taken by increasing shift (ties by
// index); a row that reduces to zero against the earlier independent rows
// gives the constant basis row e_i - sum c_j e_j (its combination), an
// independent row gives x e_i.  That matrix is the s-Popov basis at order 1.
//
// Instead of forming P F at every round, G = P F (the residual series) is
// updated with the same row operations as P; its coefficient k is R.  These
// leaves are small sequential eliminations (orders up to a few dozen); the
// polynomial products of PM-Basis above them run on the GPU.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/pm.h"
#include "pm_plan.h"

namespace {

typedef unsigned __int128 u128;

// Arithmetic mod p.  For p < 2^32 products fit 64 bits and are reduced with
// Barrett's method (mu = floor((2^64-1)/p)); sums of products are kept in
// 128 bits and reduced once.
struct Field {
  uint64_t p;
  bool small;          // p < 2^32
  uint64_t mu;         // floor((2^64 - 1) / p)
  uint64_t r64;        // 2^64 mod p
  size_t batch;        // products of two residues that a 128-bit sum takes
                       // after a reduction (< p) without wrapping
  explicit Field(uint64_t q)
      : p(q), small(q < (1ull << 32)), mu(~0ull / q), r64((uint64_t)(((u128)1 << 64) % q)) {
    // each product is at most (p-1)^2; after a reduction the sum is below p,
    // so batch terms keep it below p + batch (p-1)^2 <= (batch + 1) (p-1)^2
    const u128 sq = (u128)(q - 1) * (q - 1);
    const u128 cap = sq ? ~(u128)0 / sq : ~(u128)0;
    batch = cap - 1 > (u128)SIZE_MAX ? SIZE_MAX : (size_t)(cap > 1 ? cap - 1 : 1);
  }
  uint64_t red64(uint64_t x) const {  // x mod p, p < 2^32
    const uint64_t qt = (uint64_t)(((u128)x * mu) >> 64);
    uint64_t r = x - qt * p;
    while (r >= p) r -= p;
    return r;
  }
  uint64_t red128(u128 x) const {
    if (!small) return (uint64_t)(x % p);
    const uint64_t hi = red64((uint64_t)(x >> 64)), lo = red64((uint64_t)x);
    return add(red64(hi * r64), lo);
  }
  uint64_t add(uint64_t a, uint64_t b) const { uint64_t s = a + b; return s >= p ? s - p : s; }
  uint64_t sub(uint64_t a, uint64_t b) const { return a >= b ? a - b : a + p - b; }
  uint64_t mul(uint64_t a, uint64_t b) const {
    return small ? red64(a * b) : (uint64_t)((u128)a * b % p);
  }
  uint64_t inv(uint64_t a) const { return pm::powmod_u64(a, p - 2, p); }
};

const int64_t kNoDeg = INT64_MIN / 4;

// rdeg_s(P)_i = max_j deg(P_ij) + s_j over nonzero entries; P is (D, m, m).
void row_degrees(const std::vector<uint64_t>& P, int D, int m, const int64_t* s,
                 int64_t* out) {
  for (int i = 0; i < m; ++i) {
    int64_t best = kNoDeg;
    for (int j = 0; j < m; ++j) {
      for (int c = D - 1; c >= 0; --c) {
        if (P[((size_t)c * m + i) * m + j]) {
          best = std::max(best, (int64_t)c + s[j]);
          break;
        }
      }
    }
    out[i] = best;
  }
}

}  // namespace

static pm_status mbasis_impl(uint64_t p, int32_t m, int32_t n, int32_t sigma, const uint64_t* F,
                             const int64_t* shift, uint64_t* Pout, int64_t* rdeg_out) {
  const Field K(p);
  pm::alloc_point();
  const int D = sigma + 1;                       // coefficients of P (degree <= sigma)
  std::vector<uint64_t> P((size_t)D * m * m, 0), G((size_t)sigma * m * n, 0);
  for (int i = 0; i < m; ++i) P[(size_t)i * m + i] = 1;
  for (size_t e = 0; e < G.size(); ++e) G[e] = F[e] % p;
  std::vector<int64_t> sc(shift, shift + m);
  std::vector<int> order(m);
  std::vector<uint64_t> v(n), comb(m), newP((size_t)D * m), newG((size_t)sigma * n);
  struct Pivot { int col; std::vector<uint64_t> w, cw; };
  for (int k = 0; k < sigma; ++k) {
    // M-Basis-1 on R = coefficient k of G, shift sc
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sc[a] < sc[b]; });
    std::vector<Pivot> piv;
    std::vector<int> indep;                       // rows multiplied by x
    std::vector<std::pair<int, std::vector<uint64_t>>> dep;  // (row, combination)
    for (int i : order) {
      for (int c = 0; c < n; ++c) v[c] = G[((size_t)k * m + i) * n + c];
      std::fill(comb.begin(), comb.end(), 0);
      comb[i] = 1;
      for (const Pivot& q : piv) {
        const uint64_t f = v[q.col];
        if (!f) continue;
        for (int c = 0; c < n; ++c) v[c] = K.sub(v[c], K.mul(f, q.w[c]));
        for (int j = 0; j < m; ++j) comb[j] = K.sub(comb[j], K.mul(f, q.cw[j]));
      }
      int col = -1;
      for (int c = 0; c < n && col < 0; ++c)
        if (v[c]) col = c;
      if (col < 0) {
        dep.emplace_back(i, comb);
      } else {
        const uint64_t iv = K.inv(v[col]);
        Pivot q{col, std::vector<uint64_t>(n), std::vector<uint64_t>(m)};
        for (int c = 0; c < n; ++c) q.w[c] = K.mul(v[c], iv);
        for (int j = 0; j < m; ++j) q.cw[j] = K.mul(comb[j], iv);
        piv.push_back(std::move(q));
        indep.push_back(i);
      }
    }
    // P := Q P and G := Q G.  Constant rows combine the old rows (their
    // support is on the row itself and independent rows, which are updated
    // after); independent rows are multiplied by x.
    // P has degree <= k before this round, so coefficients above k are zero
    const int dk = std::min(D, k + 1);
    std::vector<int> sup;
    std::vector<uint64_t> cf;
    for (auto& dc : dep) {
      const int i = dc.first;
      const std::vector<uint64_t>& cm = dc.second;
      sup.clear();
      cf.clear();
      for (int j = 0; j < m; ++j)
        if (cm[j]) { sup.push_back(j); cf.push_back(cm[j]); }
      const size_t ns = sup.size();
      // sum_u cf[u] X[row sup[u]][t] mod p, reduced every K.batch terms
      auto dot = [&](const std::vector<uint64_t>& X, size_t base, size_t row, size_t t) {
        u128 acc = 0;
        size_t run = 0;
        for (size_t u = 0; u < ns; ++u) {
          if (run == K.batch) { acc = K.red128(acc); run = 0; }
          acc += (u128)cf[u] * X[base + sup[u] * row + t];
          ++run;
        }
        return K.red128(acc);
      };
      for (int c = 0; c < dk; ++c)
        for (int t = 0; t < m; ++t) newP[(size_t)c * m + t] = dot(P, (size_t)c * m * m, m, t);
      for (int c = k; c < sigma; ++c)
        for (int t = 0; t < n; ++t) newG[(size_t)c * n + t] = dot(G, (size_t)c * m * n, n, t);
      for (int c = 0; c < dk; ++c)
        for (int t = 0; t < m; ++t) P[((size_t)c * m + i) * m + t] = newP[(size_t)c * m + t];
      for (int c = k; c < sigma; ++c)
        for (int t = 0; t < n; ++t) G[((size_t)c * m + i) * n + t] = newG[(size_t)c * n + t];
    }
    for (int i : indep) {
      for (int c = std::min(D - 1, dk); c >= 1; --c)
        for (int t = 0; t < m; ++t)
          P[((size_t)c * m + i) * m + t] = P[((size_t)(c - 1) * m + i) * m + t];
      for (int t = 0; t < m; ++t) P[(size_t)i * m + t] = 0;
      for (int c = sigma - 1; c >= 1; --c)
        for (int t = 0; t < n; ++t)
          G[((size_t)c * m + i) * n + t] = G[((size_t)(c - 1) * m + i) * n + t];
      for (int t = 0; t < n; ++t) G[(size_t)i * n + t] = 0;
    }
    row_degrees(P, std::min(D, k + 2), m, shift, sc.data());
  }
  memcpy(Pout, P.data(), sizeof(uint64_t) * P.size());
  memcpy(rdeg_out, sc.data(), sizeof(int64_t) * m);
  return PM_OK;
}

extern "C" pm_status pm_mbasis_host(uint64_t p, int32_t m, int32_t n, int32_t sigma,
                                    const uint64_t* F, const int64_t* shift, uint64_t* Pout,
                                    int64_t* rdeg_out) {
  if (!F || !shift || !Pout || !rdeg_out) return PM_EINVAL;
  if (m < 1 || n < 1 || sigma < 1) return PM_EINVAL;
  if (p >= (1ull << 62)) return PM_ERANGE;
  if (p < 2 || !pm::is_prime_u64(p)) return PM_EINVAL;
  try {
    return mbasis_impl(p, m, n, sigma, F, shift, Pout, rdeg_out);
  } catch (const std::bad_alloc&) {
    return PM_ENOMEM;
  }
}

// Inverse of an n x n matrix mod a prime p by Gauss-Jordan elimination with
// row pivoting: the constant term A(0)^{-1} with which Newton iteration for
// truncated inverses starts.
static pm_status matinv_impl(uint64_t p, int32_t n, const uint64_t* M, uint64_t* Minv) {
  const Field K(p);
  pm::alloc_point();
  const size_t w = 2 * (size_t)n;
  std::vector<uint64_t> a((size_t)n * w, 0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) a[i * w + j] = M[(size_t)i * n + j] % p;
    a[i * w + n + i] = 1;
  }
  for (int col = 0; col < n; ++col) {
    int piv = -1;
    for (int r = col; r < n && piv < 0; ++r)
      if (a[r * w + col]) piv = r;
    if (piv < 0) return PM_EINVAL;  // singular
    if (piv != col)
      for (size_t j = 0; j < w; ++j) std::swap(a[piv * w + j], a[col * w + j]);
    const uint64_t iv = K.inv(a[col * w + col]);
    for (size_t j = 0; j < w; ++j) a[col * w + j] = K.mul(a[col * w + j], iv);
    for (int r = 0; r < n; ++r) {
      const uint64_t f = a[r * w + col];
      if (r == col || !f) continue;
      for (size_t j = 0; j < w; ++j) a[r * w + j] = K.sub(a[r * w + j], K.mul(f, a[col * w + j]));
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Minv[(size_t)i * n + j] = a[i * w + n + j];
  return PM_OK;
}

extern "C" pm_status pm_matinv_host(uint64_t p, int32_t n, const uint64_t* M, uint64_t* Minv) {
  if (!M || !Minv || n < 1) return PM_EINVAL;
  if (p >= (1ull << 62)) return PM_ERANGE;
  if (p < 2 || !pm::is_prime_u64(p)) return PM_EINVAL;
  try {
    return matinv_impl(p, n, M, Minv);
  } catch (const std::bad_alloc&) {
    return PM_ENOMEM;
  }
}
