// Plain fp32 X-stage kernel: the vector-ALU comparison path.
//
// Samples are promoted to fp32 once, when a workgroup stages them in LDS
// (the paper's path promotes 8-bit samples to 32-bit floats on read, Sec. 2.4),
// and every complex multiply-accumulate is four fp32 FMAs:
//   Re += a_i a_j + b_i b_j,   Im += b_i a_j - a_i b_j.
// The work decomposition is the int8 kernel's (64x64 wave tiles, four waves
// per workgroup); inside a tile lane (u, v) owns the 8x8 complex sub-tile
// rows 8u.., columns 8v...  Sub-tiles outside the tile's kind (upper blocks of
// a diagonal tile, the other half of a half tile) are masked off.
#include "xcorr_device.h"

namespace xcorr {
namespace {

constexpr int kStep = 16;                          // samples per LDS stage
constexpr int kSlotRow = kRowBlock * 8;            // bytes of one slot at one sample (float2)
constexpr int kSampleBytes = kSlots * kSlotRow;    // 2 KiB
constexpr int kBufBytes = kStep * kSampleBytes;    // 32 KiB

__device__ __forceinline__ float nib_hi(uint32_t x, int byte)
{
    return (float)(int)__builtin_amdgcn_sbfe((int)x, 8 * byte + 4, 4);
}
__device__ __forceinline__ float nib_lo(uint32_t x, int byte)
{
    return (float)(int)__builtin_amdgcn_sbfe((int)x, 8 * byte, 4);
}
__device__ __forceinline__ float sbyte(uint32_t x, int byte)
{
    return (float)(int)__builtin_amdgcn_sbfe((int)x, 8 * byte, 8);
}

// Staging: CI4 lane -> inputs 4*(q%16)..+3, samples 4*(q/16)..+3;
// CI8 lane -> input pair 2*(q%32), samples 8*(q/32)..+7.
template <int FMT>
struct Stager {
    static constexpr int kLoads = (FMT == 0) ? 4 : 8;
    uint32_t r[kLoads];
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t vofs;
    int col, s0, row_bytes, lds_slot;

    __device__ __forceinline__ void init(const LaunchArgs& a, const WaveJob& w, int lane)
    {
        lds_slot = w.stage_rb < 0 ? -1 : w.wave;
        row_bytes = a.row_bytes;
        rsrc = channel_rsrc(a, w.stage_rb, w.stage_ch);
        if (FMT == 0) { col = 4 * (lane & 15); s0 = 4 * (lane >> 4); }
        else          { col = 2 * (lane & 31); s0 = 8 * (lane >> 5); }
        const int input = (w.stage_rb < 0 ? 0 : w.stage_rb) * kRowBlock + col;
        vofs = (uint32_t)s0 * (uint32_t)a.row_bytes + column_offset(input, a.n_inputs, FMT == 0 ? 1 : 2);
    }

    __device__ __forceinline__ void load(int t0)
    {
        const uint32_t step = (uint32_t)t0 * (uint32_t)row_bytes;
#pragma unroll
        for (int s = 0; s < kLoads; ++s)
            r[s] = load_b32(rsrc, vofs + step + (uint32_t)s * (uint32_t)row_bytes);
    }

    __device__ __forceinline__ void store(uint8_t* buf) const
    {
        if (lds_slot < 0) return;
#pragma unroll
        for (int s = 0; s < kLoads; ++s) {
            float4* p = (float4*)(buf + (s0 + s) * kSampleBytes + lds_slot * kSlotRow + col * 8);
            if (FMT == 0) {
                p[0] = make_float4(nib_hi(r[s], 0), nib_lo(r[s], 0), nib_hi(r[s], 1), nib_lo(r[s], 1));
                p[1] = make_float4(nib_hi(r[s], 2), nib_lo(r[s], 2), nib_hi(r[s], 3), nib_lo(r[s], 3));
            } else {
                p[0] = make_float4(sbyte(r[s], 0), sbyte(r[s], 1), sbyte(r[s], 2), sbyte(r[s], 3));
            }
        }
    }
};

template <int FMT>
__device__ __forceinline__ void run_tile(const LaunchArgs& a, const WaveJob& w, int lane, uint8_t* lds)
{
    Stager<FMT> st;
    st.init(a, w, lane);
    const int nk = (a.t_len + kStep - 1) / kStep;
    const int u = lane >> 3, v = lane & 7;
    const bool active = w.kind != KIND_NONE && block_on(w.kind, u >> 1, v >> 1);
    float re[8][8], im[8][8];
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int q = 0; q < 8; ++q) { re[p][q] = 0.f; im[p][q] = 0.f; }

    st.load(0);
    st.store(lds);
    __syncthreads();
    for (int k = 0; k < nk; ++k) {
        const uint8_t* cur = lds + (k & 1) * kBufBytes;
        if (k + 1 < nk) st.load((k + 1) * kStep);
        if (active) {
            for (int t = 0; t < kStep; ++t) {
                const float4* pi = (const float4*)(cur + t * kSampleBytes + w.si * kSlotRow + u * 64);
                const float4* pj = (const float4*)(cur + t * kSampleBytes + w.sj * kSlotRow + v * 64);
                float xi[16], xj[16];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float4 A = pi[q], B = pj[q];
                    xi[4 * q] = A.x; xi[4 * q + 1] = A.y; xi[4 * q + 2] = A.z; xi[4 * q + 3] = A.w;
                    xj[4 * q] = B.x; xj[4 * q + 1] = B.y; xj[4 * q + 2] = B.z; xj[4 * q + 3] = B.w;
                }
#pragma unroll
                for (int p = 0; p < 8; ++p)
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const float ar = xi[2 * p], ai = xi[2 * p + 1];
                        const float br = xj[2 * q], bi = xj[2 * q + 1];
                        re[p][q] = __builtin_fmaf(ar, br, re[p][q]);
                        re[p][q] = __builtin_fmaf(ai, bi, re[p][q]);
                        im[p][q] = __builtin_fmaf(ai, br, im[p][q]);
                        im[p][q] = __builtin_fmaf(-ar, bi, im[p][q]);
                    }
            }
        }
        if (k + 1 < nk) st.store(lds + ((k + 1) & 1) * kBufBytes);
        __syncthreads();
    }
    if (!active) return;
    const int ch = w.tile_ch;
    if (ch >= a.n_channels) return;
    const int64_t nb = (int64_t)a.n_inputs * (a.n_inputs + 1) / 2;
    const float* src = (const float*)a.src;
    float* dst = (float*)a.dst;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int i = w.rb_i * kRowBlock + 8 * u + p;
        if (i >= a.n_inputs) continue;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = w.rb_j * kRowBlock + 8 * v + q;
            if (j > i) continue;
            float xr = re[p][q], xi = im[p][q];
            const int64_t idx = ((int64_t)ch * nb + (int64_t)i * (i + 1) / 2 + j) * 2;
            if (src) {
                const float2 s = *(const float2*)(src + idx);
                xr += s.x;
                xi += s.y;
            }
            *(float2*)(dst + idx) = make_float2(xr, xi);
        }
    }
}

template <int FMT>
__global__ void __launch_bounds__(64 * kWavesF32, 1) xcorr_f32_kernel(LaunchArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kBufBytes];
    const int b = work_item_index(blockIdx.x, a.n_blocks, a.xcd_map);
    if (b >= a.n_blocks) return;
    const WaveJob w = wave_job<kWavesF32>(a, b);
    run_tile<FMT>(a, w, threadIdx.x & 63, lds);
}

}  // namespace

hipError_t launch_f32(const LaunchArgs& a, int fmt, hipStream_t s)
{
    const dim3 grid(launch_blocks(a.n_blocks, a.xcd_map)), block(64 * kWavesF32);
    if (fmt == 0) hipLaunchKernelGGL(xcorr_f32_kernel<0>, grid, block, 0, s, a);
    else          hipLaunchKernelGGL(xcorr_f32_kernel<1>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace xcorr
