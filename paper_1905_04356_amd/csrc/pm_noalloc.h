// pm_noalloc.h -- the static scratch array of pm_mul_noalloc.
#pragma once
#include <stdint.h>

namespace pm {

// Bytes of the static scratch array, and the part of it that holds the
// tables of pm_mul_noalloc; the rest is the largest workspace it offers.
constexpr uint64_t kScratchBytes = 64ull << 20;
constexpr uint64_t kScratchTableBytes = 8ull << 20;
constexpr uint64_t kScratchWorkspaceBytes = kScratchBytes - kScratchTableBytes;

// Device address of the current device's scratch array (looked up, and its
// table slice registered as the static table pool, on the first call per
// device).  PM_EDEVICE if the lookup fails.
int noalloc_scratch(uint8_t** out);

}  // namespace pm
