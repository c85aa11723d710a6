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
    void* work;              // CI4: [n_spectra][n_inputs][cp] bytes, channel-fastest codes
    int32_t n_inputs, n_taps, n_spectra, chan_begin, n_chan, out_kind;
    int32_t cp;              // channels per work row (set by the launcher)
    int32_t m_begin, m_end;  // spectra of one launch (set by the launcher)
};

// Bytes of the work buffer the CI4 output needs.
int64_t fstage_work_bytes(int n_inputs, int64_t n_spectra, int chan_begin, int n_chan);
hipError_t launch_fstage(FstageArgs a, hipStream_t s);

}  // namespace xcorr
