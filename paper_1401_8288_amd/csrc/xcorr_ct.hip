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
// (two for CI8) of every byte.
#include "xcorr_ct.h"

#include <algorithm>

namespace xcorr {
namespace {

constexpr int kThreads = 256;
constexpr int kTileBytes = 32768;

// sign-extend the two nibbles of byte k of x into int8 (re, im)
__device__ __forceinline__ uint32_t unpack2(uint32_t x, int k)
{
    const uint32_t b = (x >> (8 * k)) & 0xFFu;
    const int re = (int)(int8_t)(uint8_t)b >> 4;
    const int im = (int)(int8_t)(uint8_t)(b << 4) >> 4;
    return ((uint32_t)re & 0xFFu) | (((uint32_t)im & 0xFFu) << 8);
}

template <int OUT>
__global__ void __launch_bounds__(kThreads) corner_turn_kernel(CornerTurnArgs a)
{
    extern __shared__ uint32_t tile[];          // [CT][ST][N / 4]
    const int b = blockIdx.x / a.n_ctiles;
    const int c0 = (blockIdx.x - b * a.n_ctiles) * a.ct;
    const int s0 = blockIdx.y * a.st;
    const int nc = min(a.ct, a.n_channels - c0);
    const int ns = min(a.st, a.spectra - s0);
    const int jw = a.inputs_per_feng >> 2;      // dwords per (f, s, c) segment
    const int nw = a.n_inputs >> 2;             // dwords per output row
    const uint32_t* in = (const uint32_t*)a.in;

    // gather: (f, s, c, w) with w fastest, then c, so that consecutive lanes
    // read consecutive dwords of one contiguous segment
    const int per_f = ns * nc * jw;
    const int total = a.n_fengines * per_f;
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        int r = idx;
        const int w = r % jw;  r /= jw;
        const int c = r % nc;  r /= nc;
        const int s = r % ns;
        const int f = r / ns;
        const bool ok = a.valid == nullptr || a.valid[(int64_t)b * a.n_fengines + f] != 0;
        uint32_t v = 0;
        if (ok) {
            const int64_t src = ((((int64_t)b * a.n_fengines + f) * a.spectra + s0 + s) * a.n_channels + c0 + c) * jw + w;
            v = in[src];
        }
        tile[(c * a.st + s) * nw + f * jw + w] = v;
    }
    __syncthreads();

    // scatter: for each channel the ns rows are contiguous in the output
    const int rows = ns * nw;
    for (int idx = threadIdx.x; idx < nc * rows; idx += kThreads) {
        const int c = idx / rows, q = idx - c * rows;
        const int s = q / nw, w = q - s * nw;
        const uint32_t v = tile[(c * a.st + s) * nw + w];
        const int64_t row = ((int64_t)(c0 + c) * a.n_time + (int64_t)b * a.spectra + s0 + s);
        if (OUT == 0) {
            ((uint32_t*)a.out)[row * nw + w] = v;
        } else {
            uint2 o;
            o.x = unpack2(v, 0) | (unpack2(v, 1) << 16);
            o.y = unpack2(v, 2) | (unpack2(v, 3) << 16);
            ((uint2*)a.out)[row * nw + w] = o;
        }
    }
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
    if (gx > 0x7fffffff) return hipErrorInvalidConfiguration;
    const int gy = (a.spectra + a.st - 1) / a.st;
    if (gy > 65535) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)gx, gy, 1);
    const size_t lds = (size_t)a.ct * a.st * row_bytes;
    if (out_format == 0) hipLaunchKernelGGL(corner_turn_kernel<0>, grid, dim3(kThreads), lds, s, a);
    else                 hipLaunchKernelGGL(corner_turn_kernel<1>, grid, dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace xcorr
