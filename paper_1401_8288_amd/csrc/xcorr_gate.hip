// Row gather for pulsar gating (Sec. 5): copies the selected time samples of
// every channel into a packed buffer.  A workgroup takes one channel and a
// run of output rows and moves them in 16-byte units (4-byte units when the
// row length is not a multiple of 16); HBM-bound, one read and one write of
// every kept byte.
#include "xcorr_gate.h"

namespace xcorr {
namespace {

constexpr int kThreads = 256;
constexpr int kUnitsPerBlock = 4096;   // 64 KB of 16-byte units per workgroup

template <typename T>
__global__ void __launch_bounds__(kThreads) gather_rows_kernel(T* out, const T* in, const int32_t* idx,
                                                               int64_t n_kept, int64_t n_time, int row_units,
                                                               int rows_per_block, int n_channels)
{
    const int64_t k0 = (int64_t)blockIdx.x * rows_per_block;
    const int nk = (int)(n_kept - k0 < rows_per_block ? n_kept - k0 : rows_per_block);
    const int units = nk * row_units;
    for (int c = blockIdx.y; c < n_channels; c += gridDim.y) {
        const T* src = in + (int64_t)c * n_time * row_units;
        T* dst = out + ((int64_t)c * n_kept + k0) * row_units;
        for (int u = threadIdx.x; u < units; u += kThreads) {
            const int r = u / row_units, q = u - r * row_units;
            dst[u] = src[(int64_t)idx[k0 + r] * row_units + q];
        }
    }
}

}  // namespace

hipError_t launch_gather_rows(void* out, const void* in, const int32_t* idx, int64_t n_kept, int64_t n_time,
                              int64_t row_bytes, int n_channels, hipStream_t s)
{
    if (n_kept <= 0 || n_channels <= 0) return hipSuccess;
    const bool wide = row_bytes % 16 == 0;
    const int64_t row_units = row_bytes / (wide ? 16 : 4);
    if (row_units <= 0 || row_units > (1 << 20)) return hipErrorInvalidValue;
    const int rows = (int)(row_units >= kUnitsPerBlock ? 1 : kUnitsPerBlock / row_units);
    const int64_t gx = (n_kept + rows - 1) / rows;
    if (gx > 0x7fffffff) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)gx, n_channels < 65535 ? n_channels : 65535);
    if (wide)
        hipLaunchKernelGGL(gather_rows_kernel<uint4>, grid, dim3(kThreads), 0, s, (uint4*)out, (const uint4*)in, idx,
                           n_kept, n_time, (int)row_units, rows, n_channels);
    else
        hipLaunchKernelGGL(gather_rows_kernel<uint32_t>, grid, dim3(kThreads), 0, s, (uint32_t*)out,
                           (const uint32_t*)in, idx, n_kept, n_time, (int)row_units, rows, n_channels);
    return hipGetLastError();
}

}  // namespace xcorr
