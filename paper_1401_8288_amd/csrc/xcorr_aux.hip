// Small HBM-bound helper kernels: zero fill and copy.
// Written as kernels (not hipMemsetAsync / hipMemcpyAsync) so that a caller
// may capture any library call into a HIP graph.
#include "xcorr_internal.h"

namespace xcorr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

__global__ void fill_zero_kernel(v4i* dst, size_t n16, uint8_t* tail, size_t n_tail)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride)
        dst[k] = v4i{0, 0, 0, 0};
    if (blockIdx.x == 0 && threadIdx.x < n_tail) tail[threadIdx.x] = 0;
}

__global__ void copy_kernel(v4i* dst, const v4i* src, size_t n16, uint8_t* tail,
                            const uint8_t* stail, size_t n_tail)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride)
        dst[k] = src[k];
    if (blockIdx.x == 0 && threadIdx.x < n_tail) tail[threadIdx.x] = stail[threadIdx.x];
}

// out[k] = (a64 ? a64[k] : 0) + (a32 ? a32[k] : 0) over n (re, im) pairs, out
// and a64 int64, a32 int32 (out may be a64).
__global__ void __launch_bounds__(256) add_i32_kernel(longlong2* out, const longlong2* a64, const int2* a32, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        longlong2 v = a64 ? a64[k] : longlong2{0, 0};
        if (a32) {
            const int2 w = a32[k];
            v.x += w.x;
            v.y += w.y;
        }
        out[k] = v;
    }
}

// Row c, t of out (out_row bytes) = row c, src(t) of in (in_row <= out_row
// bytes, src(t) = idx[t] or t) followed by zeros.  One thread per output
// dword; the input is read bytewise (its rows need no alignment).
__global__ void __launch_bounds__(256) pad_rows_kernel(uint8_t* out, int out_row, const uint8_t* in, int in_row,
                                                       int64_t in_chan_stride, const int32_t* idx, int64_t n_rows,
                                                       int n_channels)
{
    const int per_row = out_row / 4;
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_rows * per_row) return;
    const int64_t t = u / per_row;
    const int q = (int)(u - t * per_row);
    const int64_t ts = idx ? idx[t] : t;
    for (int c = blockIdx.y; c < n_channels; c += gridDim.y) {
        const uint8_t* src = in + c * in_chan_stride + ts * in_row;
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = 4 * q + b;
            if (k < in_row) v |= (uint32_t)src[k] << (8 * b);
        }
        *(uint32_t*)(out + ((int64_t)c * n_rows + t) * out_row + 4 * q) = v;
    }
}

int grid_for(size_t n)
{
    const size_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16, n_tail = bytes % 16;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n16)), dim3(256), 0, s, (v4i*)dst, n16,
                       (uint8_t*)dst + n16 * 16, n_tail);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16, n_tail = bytes % 16;
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n16)), dim3(256), 0, s, (v4i*)dst,
                       (const v4i*)src, n16, (uint8_t*)dst + n16 * 16,
                       (const uint8_t*)src + n16 * 16, n_tail);
    return hipGetLastError();
}

hipError_t launch_add_i32(void* out, const void* a64, const void* a32, size_t n_pairs, hipStream_t s)
{
    hipLaunchKernelGGL(add_i32_kernel, dim3(grid_for(n_pairs)), dim3(256), 0, s, (longlong2*)out,
                       (const longlong2*)a64, (const int2*)a32, n_pairs);
    return hipGetLastError();
}

hipError_t launch_pad_rows(uint8_t* out, int out_row, const uint8_t* in, int in_row, int64_t in_chan_stride,
                           const int32_t* idx, int64_t n_rows, int n_channels, hipStream_t s)
{
    if (n_rows <= 0 || n_channels <= 0) return hipSuccess;
    if (out_row % 4 || in_row > out_row) return hipErrorInvalidValue;
    const int64_t gx = (n_rows * (out_row / 4) + 255) / 256;
    if (gx > 0x7fffffff) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)gx, n_channels < 65535 ? n_channels : 65535);
    hipLaunchKernelGGL(pad_rows_kernel, grid, dim3(256), 0, s, out, out_row, in, in_row, in_chan_stride, idx, n_rows,
                       n_channels);
    return hipGetLastError();
}

}  // namespace xcorr
