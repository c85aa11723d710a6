// Row gather for gated accumulation: the samples of each gate are packed
// next to each other before the X-stage runs over them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xcorr {

// out[c][k][:] = in[c][idx[k]][:] for k < n_kept; rows of row_bytes bytes
// (a multiple of 4), in has n_time rows per channel.
hipError_t launch_gather_rows(void* out, const void* in, const int32_t* idx, int64_t n_kept, int64_t n_time,
                              int64_t row_bytes, int n_channels, hipStream_t s);

}  // namespace xcorr
