// Fixed per-device scratch of the no-allocation sigma entry point.
#pragma once
#include "common.h"

namespace dmrg {

// 64 MiB: the largest stage-1 workspace (one chunk) dmrg_sigma_noalloc serves.
constexpr int64_t kNoAllocScratchDoubles = (int64_t)8 << 20;

// Looks up (once per device; the device must be current) and caches the
// device address of the scratch array.
double* noalloc_scratch_init(int device);
// The cached address, or nullptr before noalloc_scratch_init on that device.
double* noalloc_scratch(int device);

}  // namespace dmrg
