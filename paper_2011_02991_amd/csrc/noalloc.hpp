// noalloc.hpp -- the fixed device scratch of the entry point that allocates
// nothing (see noalloc.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>

namespace qng {

// Size of the fixed scratch each GPU holds for the process's lifetime.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;

// Look up the device address of the scratch on `device`, which must be the
// current device; once per device (later calls return hipSuccess at once).
hipError_t noalloc_scratch_init(int device);

// The address found by noalloc_scratch_init for `device`, or nullptr.
void *noalloc_scratch(int device);

}  // namespace qng
