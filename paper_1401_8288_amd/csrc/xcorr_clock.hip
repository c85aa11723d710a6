// Shader-clock probe for measurement: one wave reads the shader cycle
// counter and the constant-rate wall clock, waits a given number of
// wall-clock ticks (bounded by an iteration cap, so the wave always ends),
// and reads both again.  Run beside a long kernel on another stream, the
// ratio of the two counts is the shader clock under that kernel's load,
// which sets the MFMA peak the kernel can reach at that moment.
#include "xcorr_clock.h"

namespace xcorr {
namespace {

constexpr int kMaxSpins = 1 << 22;

__global__ void __launch_bounds__(64) clock_probe_kernel(unsigned long long* out, long long ticks)
{
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    unsigned long long r = r0;
    for (int i = 0; i < kMaxSpins && (long long)(r - r0) < ticks; ++i) {
        __builtin_amdgcn_s_sleep(8);
        r = __builtin_amdgcn_s_memrealtime();
    }
    const unsigned long long c1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    if (threadIdx.x == 0) {
        out[0] = r0;
        out[1] = r1;
        out[2] = c0;
        out[3] = c1;
    }
}

}  // namespace

hipError_t launch_clock_probe(unsigned long long* out, long long ticks, hipStream_t s)
{
    hipLaunchKernelGGL(clock_probe_kernel, dim3(1), dim3(64), 0, s, out, ticks);
    return hipGetLastError();
}

}  // namespace xcorr
