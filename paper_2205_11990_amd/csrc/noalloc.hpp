// Fixed device scratch for callers that cannot allocate (see noalloc.hip).
#pragma once
#include "common.hpp"

namespace mpsv {

// Bytes of the scratch array (per GPU).
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;

// The current device's scratch array (device address; looked up on the
// first call on each device).  Every user on one device shares it.
double* noalloc_scratch();

}  // namespace mpsv
