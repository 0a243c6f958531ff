// pm_mbasis.hip -- Algorithm M-Basis on the device: the leaves of PM-Basis
// (Section 3, "Approximant bases"), one workgroup per instance.
//
// Round k of M-Basis takes the residual R = coefficient k of G = P F, the
// s'-Popov approximant basis Q of R at order 1 (M-Basis-1), and sets
// P := Q P, G := Q G, s' := rdeg_s(P).  M-Basis-1: rows are taken by
// increasing shift s' (ties by index); a row that reduces to zero against
// the earlier independent rows gives the constant basis row e_i - sum c_j e_j
// (its combination), an independent row gives x e_i.
//
// The elimination runs right-looking on [R | I] in LDS: when a row becomes a
// pivot (normalised so that its first nonzero entry is 1), its column is
// cleared from every later row at once.  Each row therefore meets the pivots
// in the order they were made, with the same multipliers as a row-by-row
// elimination, so the result is the same residue for residue.  A dependent
// row's combination has support on itself (coefficient 1) and on pivot rows,
// which are updated after the dependent ones; so P_i += sum_j c_ij P_j (and
// the same for G) can run in place, each element by one thread.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pm.h"
#include "pm_profile.h"

namespace pm {
namespace {

constexpr int kMbNT = 256;

struct MbField {
  uint32_t p;
  uint64_t mu;  // floor((2^64 - 1) / p)
  __device__ uint32_t red(uint64_t x) const {
    const uint64_t qt = __umul64hi(x, mu);
    uint64_t r = x - qt * p;
    while (r >= p) r -= p;
    return (uint32_t)r;
  }
  __device__ uint32_t mul(uint32_t a, uint32_t b) const { return red((uint64_t)a * b); }
  __device__ uint32_t sub(uint32_t a, uint32_t b) const { return a >= b ? a - b : a + p - b; }
  __device__ uint32_t add(uint32_t a, uint32_t b) const {
    const uint32_t s = a + b;  // p < 2^31: no overflow
    return s >= p ? s - p : s;
  }
  __device__ uint32_t inv(uint32_t a) const {  // a^(p-2)
    uint32_t r = 1, b = a, e = p - 2;
    while (e) {
      if (e & 1) r = mul(r, b);
      b = mul(b, b);
      e >>= 1;
    }
    return r;
  }
};

// One instance: F (sigma, m, n), P (sigma + 1, m, m) written in place, shift
// and rdeg (m each), G: sigma m n words of workspace.
__global__ __launch_bounds__(kMbNT) void mbasis_kernel(uint32_t p, uint64_t mu, int m, int n,
                                                       int sigma, const uint32_t* F,
                                                       uint64_t f_stride, const int64_t* shift,
                                                       uint32_t* Pall, int64_t* rdeg_all,
                                                       uint32_t* Gall) {
  extern __shared__ uint32_t smem[];
  const MbField K{p, mu};
  const int inst = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int w = n + m;                              // [R | I] row width
  const int D = sigma + 1;
  const uint32_t* Fi = F + (size_t)inst * f_stride;
  const int64_t* s = shift + (size_t)inst * m;
  uint32_t* P = Pall + (size_t)inst * D * m * m;
  int64_t* rdeg = rdeg_all + (size_t)inst * m;
  uint32_t* G = Gall + (size_t)inst * sigma * m * n;
  // LDS: [R | I] (reused for staging rows and degrees after the
  // elimination), the dependent rows' combinations over the pivot rows, the
  // pivot multipliers, row order, flags and lists, and the shifts.
  uint32_t* W = smem;                               // m x w
  uint32_t* Cc = W + (size_t)m * w;                 // ndep x npiv <= m^2 / 4
  uint32_t* fr = Cc + (size_t)m * m / 4 + 1;        // multipliers of one pivot step
  int* ord = (int*)(fr + m);                        // rows by increasing shift
  int* dep = ord + m;                               // 1: dependent row this round
  int* pv = dep + m;                                // pivot rows, in index order
  int* dv = pv + m;                                 // dependent rows, in index order
  const size_t words = ((size_t)m * w + (size_t)m * m / 4 + 1 + 5 * (size_t)m + 1) & ~(size_t)1;
  int64_t* sc = (int64_t*)(smem + words);           // current shift s'
  int64_t* s0 = sc + m;                             // the shift s
  __shared__ int s_col, s_npiv, s_ndep;
  __shared__ uint32_t s_inv;

  for (size_t e = tid; e < (size_t)D * m * m; e += nt) {
    const int c = (int)(e / ((size_t)m * m)), ij = (int)(e % ((size_t)m * m));
    P[e] = (c == 0 && ij / m == ij % m) ? 1u : 0u;
  }
  for (size_t e = tid; e < (size_t)sigma * m * n; e += nt) G[e] = Fi[e] % p;
  for (int i = tid; i < m; i += nt) sc[i] = s0[i] = s[i];
  __syncthreads();

  for (int k = 0; k < sigma; ++k) {
    // rows ordered by (sc, index)
    for (int i = tid; i < m; i += nt) {
      int rank = 0;
      for (int j = 0; j < m; ++j) rank += sc[j] < sc[i] || (sc[j] == sc[i] && j < i);
      ord[rank] = i;
      dep[i] = 0;
    }
    // [R | I]
    for (int e = tid; e < m * w; e += nt) {
      const int i = e / w, c = e % w;
      W[e] = c < n ? G[((size_t)k * m + i) * n + c] : (c - n == i ? 1u : 0u);
    }
    __syncthreads();
    for (int t = 0; t < m; ++t) {
      const int r = ord[t];
      if (tid == 0) s_col = n;
      __syncthreads();
      for (int c = tid; c < n; c += nt)
        if (W[r * w + c]) atomicMin(&s_col, c);
      __syncthreads();
      const int col = s_col;
      if (col == n) {                               // dependent row
        if (tid == 0) dep[r] = 1;
        continue;                                   // (s_col is reset after a barrier)
      }
      if (tid == 0) s_inv = K.inv(W[r * w + col]);
      __syncthreads();
      const uint32_t iv = s_inv;
      for (int c = tid; c < w; c += nt) W[r * w + c] = K.mul(W[r * w + c], iv);
      for (int u = t + 1 + tid; u < m; u += nt) fr[u] = W[ord[u] * w + col];
      __syncthreads();
      // clear the pivot column from the later rows (fr holds their multipliers)
      for (int e = tid; e < (m - t - 1) * w; e += nt) {
        const int u = t + 1 + e / w, c = e % w;
        const uint32_t f = fr[u];
        if (f) {
          const int r2 = ord[u];
          W[r2 * w + c] = K.sub(W[r2 * w + c], K.mul(f, W[r * w + c]));
        }
      }
      __syncthreads();
    }
    // pivot and dependent rows, and the dependent rows' coefficients over
    // the pivot rows (their coefficient on themselves is 1)
    if (tid == 0) {
      int np = 0, nd = 0;
      for (int i = 0; i < m; ++i) {
        if (dep[i]) dv[nd++] = i;
        else pv[np++] = i;
      }
      s_npiv = np;
      s_ndep = nd;
    }
    __syncthreads();
    const int npiv = s_npiv, ndep = s_ndep;
    for (int e = tid; e < ndep * npiv; e += nt)
      Cc[e] = W[dv[e / npiv] * w + n + pv[e % npiv]];
    __syncthreads();
    // P_i += sum_j c_ij P_j for dependent i, pivot j: coefficients below dk
    // (P has degree <= k), the pivot rows of one coefficient staged in LDS
    const int dk = k + 1 < D ? k + 1 : D;
    if (ndep > 0 && npiv > 0) {
      for (int c = 0; c < dk; ++c) {
        uint32_t* Pc = P + (size_t)c * m * m;
        for (int e = tid; e < npiv * m; e += nt) W[e] = Pc[(size_t)pv[e / m] * m + e % m];
        __syncthreads();
        for (int e = tid; e < ndep * m; e += nt) {
          const int d = e / m, tcol = e % m;
          uint32_t acc = Pc[(size_t)dv[d] * m + tcol];
          for (int u = 0; u < npiv; ++u) acc = K.add(acc, K.mul(Cc[d * npiv + u], W[u * m + tcol]));
          Pc[(size_t)dv[d] * m + tcol] = acc;
        }
        __syncthreads();
      }
      // G likewise for coefficients k..sigma-1
      for (int c = k; c < sigma; ++c) {
        uint32_t* Gc = G + (size_t)c * m * n;
        for (int e = tid; e < npiv * n; e += nt) W[e] = Gc[(size_t)pv[e / n] * n + e % n];
        __syncthreads();
        for (int e = tid; e < ndep * n; e += nt) {
          const int d = e / n, tcol = e % n;
          uint32_t acc = Gc[(size_t)dv[d] * n + tcol];
          for (int u = 0; u < npiv; ++u) acc = K.add(acc, K.mul(Cc[d * npiv + u], W[u * n + tcol]));
          Gc[(size_t)dv[d] * n + tcol] = acc;
        }
        __syncthreads();
      }
    }
    // pivot rows times x
    for (int e = tid; e < npiv * m; e += nt) {
      const int i = pv[e / m], tcol = e % m;
      const int top = dk < D - 1 ? dk : D - 1;
      for (int c = top; c >= 1; --c)
        P[((size_t)c * m + i) * m + tcol] = P[((size_t)(c - 1) * m + i) * m + tcol];
      P[(size_t)i * m + tcol] = 0;
    }
    for (int e = tid; e < npiv * n; e += nt) {
      const int i = pv[e / n], tcol = e % n;
      for (int c = sigma - 1; c >= 1; --c)
        G[((size_t)c * m + i) * n + tcol] = G[((size_t)(c - 1) * m + i) * n + tcol];
      G[(size_t)i * n + tcol] = 0;
    }
    __syncthreads();
    // s' = rdeg_s(P) with the original shift s, over coefficients < k + 2:
    // the degree of every entry into LDS, then a maximum per row
    const int dd = k + 2 < D ? k + 2 : D;
    int* deg = (int*)W;                               // m x m
    for (int e = tid; e < m * m; e += nt) {
      int dg = -1;
      for (int c = dd - 1; c >= 0; --c)
        if (P[(size_t)c * m * m + e]) {
          dg = c;
          break;
        }
      deg[e] = dg;
    }
    __syncthreads();
    for (int i = tid; i < m; i += nt) {
      int64_t best = INT64_MIN / 4;
      for (int j = 0; j < m; ++j)
        if (deg[i * m + j] >= 0 && (int64_t)deg[i * m + j] + s0[j] > best)
          best = (int64_t)deg[i * m + j] + s0[j];
      sc[i] = best;
    }
    __syncthreads();
  }
  for (int i = tid; i < m; i += nt) rdeg[i] = sc[i];
}

// [R | I], the combinations, the multipliers, the order, flags and row lists
// in 32-bit words (rounded up to an even count), then two shifts in 64-bit
// words.
size_t mbasis_lds_bytes(int m, int n) {
  const size_t words =
      ((size_t)m * (n + m) + (size_t)m * m / 4 + 1 + 5 * (size_t)m + 1) & ~(size_t)1;
  return 4 * words + 16 * (size_t)m;
}

}  // namespace
}  // namespace pm

extern "C" {

pm_status pm_mbasis_workspace_bytes(int32_t count, int32_t m, int32_t n, int32_t sigma,
                                    uint64_t* out) {
  if (!out || count < 1 || m < 1 || n < 1 || sigma < 1) return PM_EINVAL;
  if (pm::mbasis_lds_bytes(m, n) > 160 * 1024) return PM_EUNSUPPORTED;
  *out = 4ull * count * sigma * m * n;
  return PM_OK;
}

pm_status pm_mbasis_u32(uint32_t p, int32_t count, int32_t m, int32_t n, int32_t sigma,
                        const uint32_t* F, uint64_t f_stride, const int64_t* shift, uint32_t* P,
                        int64_t* rdeg, void* workspace, uint64_t workspace_bytes, void* stream) {
  if (!F || !shift || !P || !rdeg || count < 1 || m < 1 || n < 1 || sigma < 1)
    return PM_EINVAL;
  if (p < 2 || p >= (1u << 31)) return PM_ERANGE;
  if (f_stride < (uint64_t)sigma * m * n) return PM_EINVAL;
  uint64_t need = 0;
  const pm_status st = pm_mbasis_workspace_bytes(count, m, n, sigma, &need);
  if (st != PM_OK) return st;
  if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 255))
    return PM_EWORKSPACE;
  const size_t lds = pm::mbasis_lds_bytes(m, n);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)pm::mbasis_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return PM_EDEVICE;
  const uint64_t mu = ~0ull / p;
  const hipError_t e =
      pm::launch(pm::mbasis_kernel, dim3((unsigned)count), dim3(pm::kMbNT), lds,
                 (hipStream_t)stream, p, mu, (int)m, (int)n, (int)sigma, F, f_stride, shift, P,
                 rdeg, (uint32_t*)workspace);
  return e == hipSuccess ? PM_OK : PM_EDEVICE;
}

}  // extern "C"
