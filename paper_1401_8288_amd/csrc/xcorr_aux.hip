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

}  // namespace xcorr
