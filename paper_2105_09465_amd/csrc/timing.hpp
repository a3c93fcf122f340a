// Opt-in event timing of the kernel-matrix product launches.
#pragma once

#include <hip/hip_runtime.h>

namespace gpl {

// Record a start event on `stream` when timing is enabled (nullptr otherwise).
hipEvent_t timing_begin(hipStream_t stream);
// Record the matching stop event.
void timing_end(hipEvent_t begin, hipStream_t stream);

}  // namespace gpl
