// Corner-turn kernel interface (packet order -> X-stage order).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xcorr {

struct CornerTurnArgs {
    const uint8_t* in;             // [block][F][S][C][J] bytes
    const uint8_t* valid;          // [block][F], 0 = lost packet; may be null
    void* out;                     // [C][T][F*J] (CI4) or [C][T][F*J][2] (CI8)
    int32_t n_blocks, n_fengines, inputs_per_feng, n_channels, spectra, n_inputs;
    int64_t n_time;
    int32_t ct, st, n_ctiles;      // tile (set by the launcher)
};

hipError_t launch_corner_turn(CornerTurnArgs a, int out_format, hipStream_t s);

}  // namespace xcorr
