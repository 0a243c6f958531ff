// pm_vdm_tables.cpp -- Vandermonde matrices for evaluation at the points
// 0, 1, ..., N-1 (N = 2d - 1) and interpolation back, mod a prime p >= N.
//
// V (N x d): V[i][c] = i^c.  W (N x N) = inverse of the square Vandermonde
// matrix, from the Lagrange basis: with M(x) = prod_j (x - j) and
// Q_i = M / (x - i), the interpolant of values y_i has coefficients
// sum_i y_i Q_i[c] / Q_i(i), so W[c][i] = Q_i[c] / Q_i(i).  Both are built
// on the host in O(N^2) operations and kept on the device until the process
// ends, per (device, p, d).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/pm.h"
#include "pm_plan.h"
#include "pm_vdm.h"

namespace pm {

namespace {

struct VdmEntry {
  uint32_t* V = nullptr;
  uint32_t* W = nullptr;
};
std::mutex g_vmu;
std::map<std::tuple<int, uint32_t, int>, VdmEntry> g_vdm;

uint64_t mulm(uint64_t a, uint64_t b, uint64_t p) { return a * b % p; }  // p < 2^31

}  // namespace

int get_vdm_tables(uint32_t p, int d, const uint32_t** V, const uint32_t** W) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PM_EDEVICE;
  std::lock_guard<std::mutex> lock(g_vmu);
  auto key = std::make_tuple(dev, p, d);
  auto it = g_vdm.find(key);
  if (it == g_vdm.end()) {
    const int N = 2 * d - 1;
    std::vector<uint32_t> hv, hw;
    try {
      hv.assign((size_t)N * d, 0);
      hw.assign((size_t)N * N, 0);
    } catch (const std::bad_alloc&) {
      return PM_ENOMEM;
    }
    for (int i = 0; i < N; ++i) {
      uint64_t x = 1;
      for (int c = 0; c < d; ++c) {
        hv[(size_t)i * d + c] = (uint32_t)x;
        x = mulm(x, (uint64_t)i, p);
      }
    }
    // M(x) = prod_{j<N} (x - j), coefficients M[0..N]
    std::vector<uint64_t> M(N + 1, 0), Q(N);
    M[0] = 1;
    for (int j = 0; j < N; ++j) {
      const uint64_t nj = (p - (uint64_t)j % p) % p;
      for (int c = j + 1; c >= 1; --c) M[c] = (M[c - 1] + mulm(M[c], nj, p)) % p;
      M[0] = mulm(M[0], nj, p);
    }
    for (int i = 0; i < N; ++i) {
      // Q = M / (x - i) by synthetic division: Q[c-1] = M[c] + i Q[c]
      Q[N - 1] = M[N];
      for (int c = N - 1; c >= 1; --c) Q[c - 1] = (M[c] + mulm((uint64_t)i, Q[c], p)) % p;
      uint64_t den = 0;  // Q(i) by Horner
      for (int c = N - 1; c >= 0; --c) den = (mulm(den, (uint64_t)i, p) + Q[c]) % p;
      const uint64_t inv = powmod_u64(den, p - 2, p);
      for (int c = 0; c < N; ++c) hw[(size_t)c * N + i] = (uint32_t)mulm(Q[c], inv, p);
    }
    VdmEntry e;
    if (hipMalloc((void**)&e.V, hv.size() * 4) != hipSuccess) return PM_ENOMEM;
    if (hipMalloc((void**)&e.W, hw.size() * 4) != hipSuccess) {
      (void)hipFree(e.V);
      return PM_ENOMEM;
    }
    if (hipMemcpy(e.V, hv.data(), hv.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(e.W, hw.data(), hw.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(e.V);
      (void)hipFree(e.W);
      return PM_EDEVICE;
    }
    it = g_vdm.emplace(key, e).first;
  }
  *V = it->second.V;
  *W = it->second.W;
  return PM_OK;
}

}  // namespace pm
