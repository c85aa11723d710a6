// Selective dump of the plan accumulator by 64 x 64 tile (baseline-dependent
// integration).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xcorr {

// For every channel and baseline (i >= j) whose tile (i / 64, j / 64) is
// selected (sel[ti (ti + 1) / 2 + tj] != 0): out = acc (or 0 if !acc_valid)
// plus acc32 (int32 pairs, if non-null; elem 16 only) and, if reset, both
// are zeroed there.  elem = bytes of one (re, im) pair (16 or 8).
hipError_t launch_dump_tiles(void* out, void* acc, int acc_valid, void* acc32, const uint8_t* sel, int n_inputs,
                             int n_channels, int elem, int reset, hipStream_t s);

}  // namespace xcorr
