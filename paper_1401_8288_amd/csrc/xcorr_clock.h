// Shader-clock probe (measurement support).
#pragma once

#include <hip/hip_runtime.h>

namespace xcorr {

// out[0..3] = wall-clock ticks at start and end, shader cycles at start and
// end, of one wave that waits `ticks` wall-clock ticks (at most 2^22 polls).
hipError_t launch_clock_probe(unsigned long long* out, long long ticks, hipStream_t s);

}  // namespace xcorr
