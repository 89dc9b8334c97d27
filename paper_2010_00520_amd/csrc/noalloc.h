// Fixed device scratch of the allocation-free translation entry point.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "tfmm.h"

namespace tfmm {

// Size of the fixed scratch array (per device).  The first 256 bytes hold the
// work counters of the persistent launches, the rest the translation scratch.
constexpr size_t kNoAllocScratchBytes = TFMM_NOALLOC_SCRATCH_BYTES;
constexpr size_t kNoAllocCounterBytes = 256;

// Look up the device address of `device`'s copy of the array; `device` must be
// current.  Idempotent; thread-safe.
hipError_t noalloc_scratch_init(int device);
// The address found by noalloc_scratch_init for `device`, or NULL.
void* noalloc_scratch(int device);

}  // namespace tfmm
