// Selective dump by tile: baseline-dependent integration (Sec. 5: dumping
// short baselines less often than long ones).  One thread per baseline of a
// row (i) of a channel; rows of tiles that are not selected do nothing.
#include "xcorr_tiles.h"

#include <type_traits>

namespace xcorr {
namespace {

// acc32 (int64 plans of the int8 path): the plan's int32 accumulator of
// the samples since its last fold, added to acc and reset with it.
template <int ELEM>
__global__ void __launch_bounds__(256) dump_tiles_kernel(void* out, void* acc, int acc_valid, int2* acc32,
                                                         const uint8_t* sel, int n_inputs, int n_channels, int reset)
{
    typedef typename std::conditional<ELEM == 16, longlong2, float2>::type T;
    const int i = blockIdx.x;
    const int64_t nb = (int64_t)n_inputs * (n_inputs + 1) / 2;
    const int ti = i >> 6;
    for (int c = blockIdx.y; c < n_channels; c += gridDim.y)
    for (int j = threadIdx.x; j <= i; j += 256) {
        const int64_t row0 = (int64_t)c * nb + (int64_t)i * (i + 1) / 2;
        const int tj = j >> 6;
        if (!sel[ti * (ti + 1) / 2 + tj]) continue;
        T* a = (T*)acc + row0 + j;
        T v;
        if (acc_valid) {
            v = *a;
            if (reset) *a = T{};
        } else {
            v = T{};
        }
        if constexpr (ELEM == 16) {
            if (acc32) {
                int2* b = acc32 + row0 + j;
                const int2 w = *b;
                v.x += w.x;
                v.y += w.y;
                if (reset) *b = int2{0, 0};
            }
        }
        ((T*)out)[row0 + j] = v;
    }
}

}  // namespace

hipError_t launch_dump_tiles(void* out, void* acc, int acc_valid, void* acc32, const uint8_t* sel, int n_inputs,
                             int n_channels, int elem, int reset, hipStream_t s)
{
    const dim3 grid(n_inputs, n_channels < 65535 ? n_channels : 65535);
    if (elem == 16)
        hipLaunchKernelGGL(dump_tiles_kernel<16>, grid, dim3(256), 0, s, out, acc, acc_valid, (int2*)acc32, sel,
                           n_inputs, n_channels, reset);
    else
        hipLaunchKernelGGL(dump_tiles_kernel<8>, grid, dim3(256), 0, s, out, acc, acc_valid, (int2*)nullptr, sel,
                           n_inputs, n_channels, reset);
    return hipGetLastError();
}

}  // namespace xcorr
