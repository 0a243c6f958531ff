// pm_tables.hip -- kernels that fill the device tables in place, on the
// stream of the call that first needs them (no host copies).
//
// Twiddles: for each pass of a transform (pass structure of make_pass_plan)
// and each stage v of the pass, the butterflies at lower index j + u S use
// w^e with e = (j + u S) 2^(logL - s - v - 1) (s = log2 S); entries are
// stored slot-major, (w^e, floor(w^e 2^32 / q)) for Shoup's multiplication,
// forward (w) then inverse (w^-1).
//
// Vandermonde (evaluation at 0 .. N-1, N = 2d - 1; Section 2 of Hyun,
// Neiger, Schost, "Polynomial matrix multiplication", the Vandermonde
// variant): V[i][c] = i^c; W = V_N^{-1} from the Lagrange basis: with
// M(x) = prod_{j<N} (x - j) and Q_i = M / (x - i), W[c][i] = Q_i[c] / Q_i(i),
// where Q_i(i) = prod_{j != i} (i - j) = i! (N-1-i)! (-1)^(N-1-i).
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

struct TwFill {
  uint32_t q, w, winv;
  int logL, npass;
  int stride_log[kMaxPasses];
  uint32_t tw_off[kMaxPasses];
  uint32_t count;  // entries per direction (>= 1)
  Tw* dst;
};

__global__ __launch_bounds__(256) void fill_twiddles_kernel(TwFill f) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= f.count) return;
  if (f.npass == 0) {  // length 1: no butterflies, one unused entry
    f.dst[idx] = Tw{0, 0};
    f.dst[f.count + idx] = Tw{0, 0};
    return;
  }
  int i = 0;
  while (i + 1 < f.npass && f.tw_off[i + 1] <= idx) ++i;
  const int s = f.stride_log[i];
  const uint32_t local = idx - f.tw_off[i];
  const uint32_t slot = local >> s, j = local & ((1u << s) - 1);
  const int v = 31 - __clz(slot + 1);
  const uint32_t u = slot + 1 - (1u << v);
  const uint64_t e = (uint64_t)(j + (u << s)) << (f.logL - s - v - 1);
  const uint32_t a = powm(f.w, e, f.q), b = powm(f.winv, e, f.q);
  f.dst[idx] = Tw{a, (uint32_t)(((uint64_t)a << 32) / f.q)};
  f.dst[f.count + idx] = Tw{b, (uint32_t)(((uint64_t)b << 32) / f.q)};
}

// One workgroup: M's N + 1 coefficients (two LDS buffers, one barrier per
// factor) and the factorials 0! .. (N-1)!, into work[0 .. N] and
// work[N + 1 .. 2N].
constexpr int kVdmNT = 1024;
__global__ __launch_bounds__(kVdmNT) void vdm_poly_kernel(uint32_t p, int N, uint32_t* work) {
  extern __shared__ uint32_t sm[];
  uint32_t* a = sm;
  uint32_t* b = sm + (N + 1);
  for (int c = threadIdx.x; c <= N; c += kVdmNT) a[c] = c == 0 ? 1 % p : 0;
  __syncthreads();
  for (int j = 0; j < N; ++j) {
    // (x - j) * a, degree j -> j + 1
    const uint32_t nj = (p - (uint32_t)(j % p)) % p;
    for (int c = threadIdx.x; c <= j + 1; c += kVdmNT) {
      const uint32_t lo = c > 0 ? a[c - 1] : 0;
      const uint32_t hi = c <= j ? mulm(a[c], nj, p) : 0;
      const uint32_t t = lo + hi;
      b[c] = t >= p ? t - p : t;
    }
    __syncthreads();
    uint32_t* t = a;
    a = b;
    b = t;
  }
  for (int c = threadIdx.x; c <= N; c += kVdmNT) work[c] = a[c];
  if (threadIdx.x == 0) {
    uint32_t f = 1 % p;
    for (int i = 0; i < N; ++i) {
      work[N + 1 + i] = f;
      f = mulm(f, (uint32_t)((i + 1) % p), p);
    }
  }
}

__global__ __launch_bounds__(256) void vdm_v_kernel(uint32_t p, int N, int d, uint32_t* V) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)N * d) return;
  const uint32_t i = (uint32_t)(idx / d), c = (uint32_t)(idx % d);
  V[idx] = powm(i % p, c, p);
}

// Thread i: column i of W by synthetic division of M by (x - i),
// Q[c - 1] = M[c] + i Q[c] from Q[N - 1] = M[N] = 1.
__global__ __launch_bounds__(256) void vdm_w_kernel(uint32_t p, int N, const uint32_t* work,
                                                    uint32_t* W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t* M = work;
  const uint32_t* fact = work + N + 1;
  uint32_t den = mulm(fact[i], fact[N - 1 - i], p);
  if ((N - 1 - i) & 1) den = den ? p - den : 0;
  const uint32_t inv = powm(den, p - 2, p);
  const uint32_t x = (uint32_t)(i % p);
  uint32_t q = M[N] % p;
  W[(size_t)(N - 1) * N + i] = mulm(q, inv, p);
  for (int c = N - 1; c >= 1; --c) {
    q = (uint32_t)(((uint64_t)x * q + M[c]) % p);
    W[(size_t)(c - 1) * N + i] = mulm(q, inv, p);
  }
}

}  // namespace

int launch_fill_twiddles(const TwKey& key, uint32_t w, uint32_t winv, Tw* dst, hipStream_t s) {
  const PassPlan PP = make_pass_plan(key.logL, key.split, key.maxr);
  TwFill f{};
  f.q = key.q;
  f.w = w;
  f.winv = winv;
  f.logL = key.logL;
  f.npass = PP.npass;
  for (int i = 0; i < PP.npass; ++i) {
    f.stride_log[i] = PP.stride_log[i];
    f.tw_off[i] = PP.tw_off[i];
  }
  f.count = PP.tw_count ? PP.tw_count : 1;
  f.dst = dst;
  return launch(fill_twiddles_kernel, dim3((f.count + 255) / 256), dim3(256), 0, s, f);
}

int launch_fill_vdm(uint32_t p, int d, uint32_t* V, uint32_t* W, uint32_t* work,
                    hipStream_t s) {
  const int N = 2 * d - 1;
  int st = launch(vdm_poly_kernel, dim3(1), dim3(kVdmNT), 8 * (size_t)(N + 1), s, p, N, work);
  if (st != hipSuccess) return st;
  const uint64_t nv = (uint64_t)N * d;
  st = launch(vdm_v_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, p, N, d, V);
  if (st != hipSuccess) return st;
  return launch(vdm_w_kernel, dim3((N + 255) / 256), dim3(256), 0, s, p, N,
                (const uint32_t*)work, W);
}

}  // namespace pm
