// Corner turn on the GPU: F-engine packet order -> X-stage input order.
//
// The X-stage input of a GPU is assembled from packets that each carry, for
// one F-engine, the GPU's channels x that F-engine's inputs for a few
// consecutive spectra (Sec. 2.4 and its packet-format figure); capture places
// them by sequence number and F-engine.  Completing the corner turn means
// putting the inputs of all F-engines of one channel and time next to each
// other, and the paper's unpacker also pads 4-bit samples to 8 bits.  Lost
// packets leave zeros.
//
//   in   [block][F][S][C][J]   bytes (4+4-bit samples)
//   out  [C][block*S + s][F*J] bytes (CI4)  or  [..][F*J][2] int8 (CI8)
//
// The kernel is a tiled transpose through LDS: a workgroup takes one block,
// a run of CT channels and a run of ST spectra, reads the F x ST segments of
// CT*J contiguous bytes, and writes for each channel ST rows of F*J bytes,
// which are contiguous in the output.  HBM-bound: one read and one write
// (two for CI8) of every byte.  Data move in units of U bytes (16 when
// J % 16 == 0, else 4), eight units per thread in flight; in LDS the unit
// u of tile row (c, s) sits at (u + c) mod (units per row), so that the
// gather's writes, which step through channels, spread over the banks.
#include "xcorr_ct.h"

#include <algorithm>

namespace xcorr {
namespace {

constexpr int kThreads = 256;
constexpr int kTileBytes = 32768;
constexpr int kBatch = 8;                       // units per thread in flight

template <int U>
struct Unit;
template <>
struct Unit<16> {
    typedef uint4 T;
    static __device__ __forceinline__ T zero() { return make_uint4(0, 0, 0, 0); }
};
template <>
struct Unit<4> {
    typedef uint32_t T;
    static __device__ __forceinline__ T zero() { return 0u; }
};

// sign-extend the nibbles of 4 packed samples into 4 (re, im) int8 pairs
__device__ __forceinline__ uint2 unpack4(uint32_t x)
{
    uint32_t r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t b = (x >> (8 * k)) & 0xFFu;
        const int re = (int)(int8_t)(uint8_t)b >> 4;
        const int im = (int)(int8_t)(uint8_t)(b << 4) >> 4;
        r[k] = ((uint32_t)re & 0xFFu) | (((uint32_t)im & 0xFFu) << 8);
    }
    return make_uint2(r[0] | (r[1] << 16), r[2] | (r[3] << 16));
}

template <int U, int OUT>
__device__ __forceinline__ void put(void* out, int64_t unit, typename Unit<U>::T v)
{
    if constexpr (OUT == 0) {
        ((typename Unit<U>::T*)out)[unit] = v;
    } else if constexpr (U == 16) {
        const uint2 a = unpack4(v.x), b = unpack4(v.y), c = unpack4(v.z), d = unpack4(v.w);
        uint4* o = (uint4*)out + 2 * unit;
        o[0] = make_uint4(a.x, a.y, b.x, b.y);
        o[1] = make_uint4(c.x, c.y, d.x, d.y);
    } else {
        ((uint2*)out)[unit] = unpack4(v);
    }
}

template <int U, int OUT>
__global__ void __launch_bounds__(kThreads) corner_turn_kernel(CornerTurnArgs a)
{
    typedef typename Unit<U>::T T;
    extern __shared__ uint4 lds_raw[];
    T* tile = (T*)lds_raw;                       // [CT][ST][N / U], rotated
    const int b = blockIdx.x / a.n_ctiles;
    const int c0 = (blockIdx.x - b * a.n_ctiles) * a.ct;
    const int s0 = blockIdx.y * a.st;
    const int nc = min(a.ct, a.n_channels - c0);
    const int ns = min(a.st, a.spectra - s0);
    const int ju = a.inputs_per_feng / U;        // units per (f, s, c) segment
    const int nu = a.n_inputs / U;               // units per row
    const T* in = (const T*)a.in;

    // gather: unit index (f, s, c, w), w fastest: consecutive lanes read one
    // contiguous segment of nc * ju units
    const int total = a.n_fengines * ns * nc * ju;
    for (int i0 = threadIdx.x; i0 < total; i0 += kThreads * kBatch) {
        T v[kBatch];
        int dst[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int idx = i0 + k * kThreads;
            dst[k] = -1;
            v[k] = Unit<U>::zero();
            if (idx < total) {
                int r = idx;
                const int w = r % ju;  r /= ju;
                const int c = r % nc;  r /= nc;
                const int s = r % ns;
                const int f = r / ns;
                int pos = f * ju + w + c % nu;
                pos -= pos >= nu ? nu : 0;
                dst[k] = (c * a.st + s) * nu + pos;
                if (a.valid == nullptr || a.valid[(int64_t)b * a.n_fengines + f] != 0)
                    v[k] = in[((((int64_t)b * a.n_fengines + f) * a.spectra + s0 + s) * a.n_channels + c0 + c) * ju + w];
            }
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
            if (dst[k] >= 0) tile[dst[k]] = v[k];
    }
    __syncthreads();

    // scatter: for each channel the ns rows are contiguous in the output
    const int rows = ns * nu;
    const int total_out = nc * rows;
    for (int i0 = threadIdx.x; i0 < total_out; i0 += kThreads * kBatch) {
        T v[kBatch];
        int64_t dst[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int idx = i0 + k * kThreads;
            dst[k] = -1;
            v[k] = Unit<U>::zero();
            if (idx < total_out) {
                const int c = idx / rows, q = idx - c * rows;
                const int s = q / nu, w = q - s * nu;
                int pos = w + c % nu;
                pos -= pos >= nu ? nu : 0;
                v[k] = tile[(c * a.st + s) * nu + pos];
                dst[k] = ((int64_t)(c0 + c) * a.n_time + (int64_t)b * a.spectra + s0 + s) * nu + w;
            }
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
            if (dst[k] >= 0) put<U, OUT>(a.out, dst[k], v[k]);
    }
}

template <int U>
hipError_t launch_unit(const CornerTurnArgs& a, dim3 grid, size_t lds, int out_format, hipStream_t s)
{
    if (out_format == 0) hipLaunchKernelGGL((corner_turn_kernel<U, 0>), grid, dim3(kThreads), lds, s, a);
    else                 hipLaunchKernelGGL((corner_turn_kernel<U, 1>), grid, dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_corner_turn(CornerTurnArgs a, int out_format, hipStream_t s)
{
    // tile: as many channels as fit in kTileBytes with all spectra of the
    // block, else one channel and as many spectra as fit
    const int64_t row_bytes = a.n_inputs;
    if ((int64_t)a.spectra * row_bytes <= kTileBytes) {
        a.st = a.spectra;
        a.ct = (int)std::min<int64_t>(a.n_channels, kTileBytes / ((int64_t)a.spectra * row_bytes));
    } else {
        a.ct = 1;
        a.st = (int)std::max<int64_t>(1, kTileBytes / row_bytes);
    }
    a.n_ctiles = (a.n_channels + a.ct - 1) / a.ct;
    const int64_t gx = (int64_t)a.n_ctiles * a.n_blocks;
    const int gy = (a.spectra + a.st - 1) / a.st;
    if (gx > 0x7fffffff || gy > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)gx, gy, 1);
    const size_t lds = (size_t)a.ct * a.st * row_bytes;
    return a.inputs_per_feng % 16 == 0 ? launch_unit<16>(a, grid, lds, out_format, s)
                                       : launch_unit<4>(a, grid, lds, out_format, s);
}

}  // namespace xcorr
