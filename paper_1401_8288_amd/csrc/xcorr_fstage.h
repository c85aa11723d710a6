// F-stage kernel interface (ADC samples -> requantised channels in X-stage order).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xcorr {

struct FstageArgs {
    const int8_t* adc;       // [n_inputs][adc_stride] real samples
    int64_t adc_stride;      // bytes between inputs (even)
    const float* coeff;      // [n_taps][8192] prototype filter
    const float* gain;       // [n_inputs][n_chan]
    void* out;               // CI4: [n_chan][n_spectra][n_inputs] bytes; F32: [..][2] floats
    int32_t n_inputs, n_taps, n_spectra, chan_begin, n_chan, out_kind;
};

hipError_t launch_fstage(const FstageArgs& a, hipStream_t s);

}  // namespace xcorr
