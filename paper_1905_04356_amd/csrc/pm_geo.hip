// pm_geo.hip -- kernels of the evaluation and interpolation at a geometric
// progression 1, a, a^2, ..., a^(N-1) (Section 2, "Polynomial
// multiplication": with an element of order at least N both take O(M(N))
// operations, the method of Bostan and Schost; used for general primes in
// "Polynomial matrix multiplication").
//
// With C2(t) = t (t - 1) / 2, i c = C2(i + c) - C2(i) - C2(c), so
//   f(a^i) = a^-C2(i) sum_c (f_c a^-C2(c)) a^C2(i + c),
// a middle product with the chirp a^C2(t).  Interpolation: with
// Q(x) = prod_j (x - a^j) and w_i = v_i / Q'(a^i), the polynomial is
// (Q S) mod x^N for the power series S = sum_i w_i / (x - a^i), whose
// coefficients s_k = -sum_i w_i a^-i(k+1) are again a chirp transform (base
// a^-1), and (Q S) mod x^N is a truncated product.  The products run through
// the library's transforms; these kernels make the tables and scale rows.
#include "pm_profile.h"
#include "pm_tables.h"

namespace pm {

namespace {

__device__ __forceinline__ uint32_t mulm(uint32_t a, uint32_t b, uint32_t q) {
  return (uint32_t)((uint64_t)a * b % q);
}

__device__ uint32_t powm(uint32_t b, uint64_t e, uint32_t q) {
  uint32_t r = 1 % q;
  while (e) {
    if (e & 1) r = mulm(r, b, q);
    b = mulm(b, b, q);
    e >>= 1;
  }
  return r;
}

// spos[t] = a^C2(t), sneg[t] = a^-C2(t) for t < T; nspos[t] = -a^C2(t) for
// t < N (exponents mod p - 1).
__global__ __launch_bounds__(256) void geo_chirp_kernel(GeoTables g) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.T) return;
  const uint64_t pm1 = g.p - 1;
  const uint64_t e = ((uint64_t)t * (t > 0 ? t - 1 : 0) / 2) % pm1;
  const uint32_t x = powm(g.a, e, g.p);
  g.spos[t] = x;
  g.sneg[t] = powm(g.a, (pm1 - e) % pm1, g.p);
  if (t < g.N) g.nspos[t] = x ? g.p - x : 0;
}

// Q(x) = prod_{j<N} (x - a^j), N + 1 coefficients, one workgroup (two LDS
// buffers, one barrier per factor).
constexpr int kQNT = 1024;
__global__ __launch_bounds__(kQNT) void geo_q_kernel(GeoTables g) {
  extern __shared__ uint32_t sm[];
  const uint32_t p = g.p;
  const int N = (int)g.N;
  uint32_t* x = sm;
  uint32_t* y = sm + (N + 1);
  for (int c = threadIdx.x; c <= N; c += kQNT) x[c] = c == 0 ? 1 : 0;
  __syncthreads();
  uint32_t aj = 1;  // a^j, the same in every thread
  for (int j = 0; j < N; ++j) {
    // (x - a^j) * x(x), degree j -> j + 1
    const uint32_t naj = aj ? p - aj : 0;
    for (int c = threadIdx.x; c <= j + 1; c += kQNT) {
      const uint32_t lo = c > 0 ? x[c - 1] : 0;
      const uint32_t hi = c <= j ? mulm(x[c], naj, p) : 0;
      const uint32_t s = lo + hi;
      y[c] = s >= p ? s - p : s;
    }
    __syncthreads();
    uint32_t* t = x;
    x = y;
    y = t;
    aj = mulm(aj, g.a, p);
  }
  for (int c = threadIdx.x; c <= N; c += kQNT) g.q[c] = x[c];
}

// fc[i] = a^(C2(i) - i) / Q'(a^i), Q'(a^i) = prod_{j != i} (a^i - a^j).
__global__ __launch_bounds__(256) void geo_weights_kernel(GeoTables g) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const uint32_t p = g.p;
  const uint32_t ai = powm(g.a, i, p);
  uint32_t prod = 1, aj = 1;
  for (uint32_t j = 0; j < g.N; ++j) {
    if (j != i) {
      const uint32_t diff = ai >= aj ? ai - aj : ai + (p - aj);
      prod = mulm(prod, diff, p);
    }
    aj = mulm(aj, g.a, p);
  }
  const uint32_t inv = powm(prod, p - 2, p);
  const uint32_t ainv_i = powm(g.a, (uint64_t)(p - 1 - (i % (p - 1))) % (p - 1), p);
  g.fc[i] = mulm(mulm(g.spos[i], ainv_i, p), inv, p);
}

// Y[r][e] = X[src][e] f[src] mod p, src = r or rows - 1 - r, e < E.
__global__ __launch_bounds__(256) void geo_scale_kernel(const uint32_t* X, uint32_t* Y,
                                                        uint32_t rows, uint64_t E,
                                                        const uint32_t* f, int reverse,
                                                        uint32_t p, uint64_t mu) {
  const uint64_t total = (uint64_t)rows * E;
  for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = idx / E, e = idx - r * E;
    const uint64_t src = reverse ? rows - 1 - r : r;
    const uint64_t x = (uint64_t)X[src * E + e] * f[src];
    uint64_t q = __umul64hi(x, mu);
    uint64_t v = x - q * p;
    if (v >= p) v -= p;
    if (v >= p) v -= p;
    Y[idx] = (uint32_t)v;
  }
}

}  // namespace

int launch_fill_geo(const GeoTables& g, hipStream_t s) {
  int st = launch(geo_chirp_kernel, dim3((g.T + 255) / 256), dim3(256), 0, s, g);
  if (st != hipSuccess) return st;
  st = launch(geo_q_kernel, dim3(1), dim3(kQNT), 8 * (size_t)(g.N + 1), s, g);
  if (st != hipSuccess) return st;
  return launch(geo_weights_kernel, dim3((g.N + 255) / 256), dim3(256), 0, s, g);
}

int launch_geo_scale(const uint32_t* X, uint32_t* Y, uint32_t rows, uint64_t E,
                     const uint32_t* f, int reverse, uint32_t p, hipStream_t s) {
  const uint64_t total = (uint64_t)rows * E;
  if (!total) return hipSuccess;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  return launch(geo_scale_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, Y, rows, E, f,
                reverse, p, (uint64_t)(~0ull / p));
}

}  // namespace pm
