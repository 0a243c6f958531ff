// pm_noalloc.hip -- the static scratch array behind pm_mul_noalloc, for
// callers that cannot allocate device memory (code under stream capture,
// serving loops, harnesses that forbid hipMalloc).
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy, at its own address, from the time the code object loads until
// the process ends.  Its first kScratchTableBytes hold the twiddle and
// Vandermonde tables of pm_mul_noalloc (a table pool of their own, registered
// once per device); the rest is the product's workspace.  In host code the
// name `scratch` is only a stand-in for the symbol: the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <new>

#include "../../include/pm.h"
#include "pm_noalloc.h"
#include "pm_tables.h"

namespace pm {

namespace {

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices] = {};

}  // namespace

int noalloc_scratch(uint8_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PM_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return PM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return PM_EDEVICE;
    }
    const int st = tables_attach_pool(kPoolStatic, p, kScratchTableBytes);
    if (st != PM_OK) return st;
    g_ptr[dev] = (uint8_t*)p;
  }
  *out = g_ptr[dev];
  return PM_OK;
}

}  // namespace pm
