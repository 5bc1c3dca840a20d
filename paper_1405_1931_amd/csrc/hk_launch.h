// Host-side entry points into the kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "hk_device.h"

namespace hk {

constexpr int kPhases = 8;
extern const char *const kPhaseNames[kPhases];

// enqueue the eight single-lattice phases on `st`; when `ev` is non-null,
// ev[0..kPhases] are recorded on `st` before each kernel and after the last;
// `pk` selects the occupancy predicate (PK_*) of the brick phase
hipError_t launch_single(const Geo &g, hipStream_t st, hipEvent_t *ev, int pk = PK_GT0);

// *p = 0 on the stream (one thread)
__global__ void k_zero_i64(int64_t *p);

}  // namespace hk
