// fp16 MFMA X-stage kernel (fp32 accumulation) for gfx950.
//
// Same tiling as the int8 kernel: per 16x16 block of complex outputs and
// 32-sample step, four v_mfma_f32_16x16x32_f16:
//   Re  += A_a(I) B_a(J) + A_b(I) B_b(J)
//   -Im += A_a(I) B_b(J) + (-A_b(I)) B_a(J)
// fp16 negation is exact, so Im needs a single accumulator; negating the
// row block's operand (one per row block and step, not one per column
// block) keeps the kernel within 256 registers, so that two workgroups
// (80 KB of LDS each) share a CU and every SIMD runs two waves: one wave's
// matrix work then covers the other's staging and barrier.  4- and 8-bit
// integers are exact in fp16 and their products are exact in fp32; the fp32
// sums are exact while every partial sum stays below 2^24.
#include "xcorr_device.h"

namespace xcorr {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef int v4i __attribute__((ext_vector_type(4)));

// LDS rows: the 64 bytes of a row's step as four 16-byte chunks, chunk c of
// row r at position (c + r / 16) % 4 of an 80-byte row.  Without the
// rotation the staging writes of a wave (rows 4 apart for 4-bit samples, 2
// apart for 8-bit ones, one chunk) fall on a quarter of the bank groups;
// with it the counted bank-conflict cycles of the 4-bit window halve.
constexpr int kStep = 32;                  // samples per LDS stage (64 bytes of fp16 per row)
constexpr int kPitch = 80;
constexpr int kPart = kRowBlock * kPitch;
constexpr int kSlotBytes = 2 * kPart;
constexpr int kBufBytes = kSlots * kSlotBytes;

// Two offset-binary values u0, u1 (< 1024, in 16-bit lanes) -> packed halves
// (1024 + u - bias) exactly: the fp16 pattern 0x6400 | u is 1024 + u.
__device__ __forceinline__ uint32_t halves(uint32_t u01, _Float16 bias)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const uint32_t bits = u01 | 0x64006400u;
    h2 h = __builtin_bit_cast(h2, bits);
    h = h - h2{bias, bias};
    return __builtin_bit_cast(uint32_t, h);
}

// Staging job: CI4 -> inputs 4*(q%16)..+3, samples 8*(q/16)..+7 of the step
// (one job per lane); CI8 -> input pair 2*(q%32), samples 8*(q/32 + 2j)..+7.
template <int FMT>
struct Stager {
    static constexpr int kJobs = (FMT == 0) ? 1 : 2;
    uint32_t r[kJobs][8];
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t vofs[kJobs];
    int row[kJobs];
    int kofs[kJobs];              // byte offset in the LDS row (2 bytes per sample)
    int row_bytes;
    int lds_slot;

    __device__ __forceinline__ void init(const LaunchArgs& a, const WaveJob& w, int lane)
    {
        lds_slot = w.stage_rb < 0 ? -1 : w.wave;
        row_bytes = a.row_bytes;
        rsrc = channel_rsrc(a, w.stage_rb, w.stage_ch);
#pragma unroll
        for (int j = 0; j < kJobs; ++j) {
            int col, tc;
            if (FMT == 0) { col = 4 * (lane & 15); tc = lane >> 4; }
            else          { col = 2 * (lane & 31); tc = (lane >> 5) + 2 * j; }
            row[j] = col;
            kofs[j] = 16 * ((tc + (col >> 4)) & 3);   // chunk tc of rows col.. (same row / 16 for all of them)
            const int input = (w.stage_rb < 0 ? 0 : w.stage_rb) * kRowBlock + col;
            vofs[j] = (uint32_t)(8 * tc) * (uint32_t)a.row_bytes +
                      column_offset(input, a.n_inputs, FMT == 0 ? 1 : 2);
        }
    }

    __device__ __forceinline__ void load(int t0)
    {
        const uint32_t step = (uint32_t)t0 * (uint32_t)row_bytes;
#pragma unroll
        for (int j = 0; j < kJobs; ++j)
#pragma unroll
            for (int s = 0; s < 8; ++s)
                r[j][s] = load_b32(rsrc, vofs[j] + step + (uint32_t)s * (uint32_t)row_bytes);
    }

    __device__ __forceinline__ void store(uint8_t* buf) const
    {
        if (lds_slot < 0) return;
        uint8_t* slot = buf + lds_slot * kSlotBytes;
#pragma unroll
        for (int j = 0; j < kJobs; ++j) {
            uint32_t o[2][4];                 // o[g][m]: samples 4g..4g+3 of byte column m
            transpose4(&r[j][0], o[0]);
            transpose4(&r[j][4], o[1]);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                v4i h;                        // 8 samples of one row as fp16
                if (FMT == 0) {
                    v4i hr;
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        // nibble n of a two's-complement value v has n ^ 8 = v + 8
                        const uint32_t x = o[g][m] ^ 0x88888888u;
                        const uint32_t lo = perm(0u, x, 0x0c010c00u);   // bytes s0, s1 -> 16-bit lanes
                        const uint32_t hi = perm(0u, x, 0x0c030c02u);   // bytes s2, s3
                        hr[2 * g] = (int)halves((lo >> 4) & 0x000F000Fu, (_Float16)1032.0f);
                        hr[2 * g + 1] = (int)halves((hi >> 4) & 0x000F000Fu, (_Float16)1032.0f);
                        h[2 * g] = (int)halves(lo & 0x000F000Fu, (_Float16)1032.0f);
                        h[2 * g + 1] = (int)halves(hi & 0x000F000Fu, (_Float16)1032.0f);
                    }
                    *(v4i*)(slot + (row[j] + m) * kPitch + kofs[j]) = hr;
                    *(v4i*)(slot + kPart + (row[j] + m) * kPitch + kofs[j]) = h;
                } else {
                    // byte columns re(2p), im(2p), re(2p+1), im(2p+1); int8 v -> v ^ 0x80 = v + 128
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        const uint32_t x = o[g][m] ^ 0x80808080u;
                        h[2 * g] = (int)halves(perm(0u, x, 0x0c010c00u), (_Float16)1152.0f);
                        h[2 * g + 1] = (int)halves(perm(0u, x, 0x0c030c02u), (_Float16)1152.0f);
                    }
                    const int part = m & 1, r_ = row[j] + (m >> 1);
                    *(v4i*)(slot + part * kPart + r_ * kPitch + kofs[j]) = h;
                }
            }
        }
    }
};

__device__ __forceinline__ v8h frag(const uint8_t* part, int blk, int lane)
{
    return *(const v8h*)(part + (16 * blk + (lane & 15)) * kPitch + 16 * (((lane >> 4) + blk) & 3));
}

__device__ __forceinline__ v8h negate(v8h x)
{
    v4i b = __builtin_bit_cast(v4i, x);
    b ^= v4i{(int)0x80008000u, (int)0x80008000u, (int)0x80008000u, (int)0x80008000u};
    return __builtin_bit_cast(v8h, b);
}

template <int FMT, int KIND>
__device__ __forceinline__ void run_tile(const LaunchArgs& a, const WaveJob& w, int lane, uint8_t* lds)
{
    Stager<FMT> st;
    st.init(a, w, lane);
    const int nk = (a.t_len + kStep - 1) / kStep;
    v4f acc_re[4][4], acc_im[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            acc_re[bi][bj] = v4f{0.f, 0.f, 0.f, 0.f};
            acc_im[bi][bj] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    const int si = w.si, sj = w.sj;

    st.load(0);
    st.store(lds);
    __syncthreads();
    for (int k = 0; k < nk; ++k) {
        uint8_t* cur = lds + (k & 1) * kBufBytes;
        if (k + 1 < nk) st.load((k + 1) * kStep);
        if (KIND != KIND_NONE) {
            const uint8_t* pI = cur + si * kSlotBytes;
            const uint8_t* pJ = cur + sj * kSlotBytes;
            v8h ia[4], ib[4], ja[4], jb[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                ia[b] = frag(pI, b, lane);
                ib[b] = frag(pI + kPart, b, lane);
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (KIND == KIND_DIAG) {
                    ja[b] = ia[b];
                    jb[b] = ib[b];
                } else if (block_on(KIND, 3, b)) {
                    ja[b] = frag(pJ, b, lane);
                    jb[b] = frag(pJ + kPart, b, lane);
                }
            }
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) {
                const v8h ibn = negate(ib[bi]);
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) {
                    if (!block_on(KIND, bi, bj)) continue;
                    acc_re[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ia[bi], ja[bj], acc_re[bi][bj], 0, 0, 0);
                    acc_re[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ib[bi], jb[bj], acc_re[bi][bj], 0, 0, 0);
                    acc_im[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ia[bi], jb[bj], acc_im[bi][bj], 0, 0, 0);
                    acc_im[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ibn, ja[bj], acc_im[bi][bj], 0, 0, 0);
                }
            }
        }
        if (k + 1 < nk) st.store(lds + ((k + 1) & 1) * kBufBytes);
        __syncthreads();
    }
    if (KIND == KIND_NONE) return;

    const int ch = w.tile_ch;
    if (ch >= a.n_channels) return;
    const int i0 = w.rb_i * kRowBlock, j0 = w.rb_j * kRowBlock;
    const int64_t nb = (int64_t)a.n_inputs * (a.n_inputs + 1) / 2;
    const float* src = (const float*)a.src;
    float* dst = (float*)a.dst;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            if (!block_on(KIND, bi, bj)) continue;
            const int j = j0 + 16 * bj + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * bi + 4 * (lane >> 4) + r;
                if (i >= a.n_inputs || j > i) continue;
                // acc_im holds -Im (0 - x also turns a -0 into +0)
                float re = acc_re[bi][bj][r], im = 0.0f - acc_im[bi][bj][r];
                const int64_t idx = ((int64_t)ch * nb + (int64_t)i * (i + 1) / 2 + j) * 2;
                if (src) {
                    const float2 s = *(const float2*)(src + idx);
                    re += s.x;
                    im += s.y;
                }
                *(float2*)(dst + idx) = make_float2(re, im);
            }
        }
}

template <int FMT>
__global__ void __launch_bounds__(64 * kWavesF16, 2) xcorr_f16_kernel(LaunchArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kBufBytes];
    const int b = work_item_index(blockIdx.x, a.n_blocks, a.xcd_map);
    if (b >= a.n_blocks) return;
    const WaveJob w = wave_job<kWavesF16>(a, b);
    const int lane = threadIdx.x & 63;
    switch (w.kind) {
    case KIND_FULL:  run_tile<FMT, KIND_FULL>(a, w, lane, lds); break;
    case KIND_DIAG:  run_tile<FMT, KIND_DIAG>(a, w, lane, lds); break;
    case KIND_HALF0: run_tile<FMT, KIND_HALF0>(a, w, lane, lds); break;
    case KIND_HALF1: run_tile<FMT, KIND_HALF1>(a, w, lane, lds); break;
    default:         run_tile<FMT, KIND_NONE>(a, w, lane, lds); break;
    }
}

}  // namespace

hipError_t launch_f16(const LaunchArgs& a, int fmt, hipStream_t s)
{
    const dim3 grid(launch_blocks(a.n_blocks, a.xcd_map)), block(64 * kWavesF16);
    if (fmt == 0) hipLaunchKernelGGL(xcorr_f16_kernel<0>, grid, block, 0, s, a);
    else          hipLaunchKernelGGL(xcorr_f16_kernel<1>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace xcorr
