// int8 MFMA X-stage kernel for gfx950.
//
// Computes, for every channel, V_ij = sum_t x_i conj(x_j) over the chunk's
// samples for the lower triangle i >= j (Sec. 1 and Sec. 2.4: the outer
// product per time and frequency, integrated on the GPU).
//
// The complex product is split into real contractions over time:
//   Re V_ij = sum a_i a_j + sum b_i b_j        (a = real part, b = imaginary)
//   Im V_ij = sum b_i a_j - sum a_i b_j
// Each sum is a 16x16x64 int8 MFMA (v_mfma_i32_16x16x64_i8) with time as the
// contraction axis.  Re uses one accumulator for both of its terms; the two
// Im terms keep their own (negating an int8 operand would not be exact for
// -128), so a 16x16 block of complex outputs costs four MFMAs and three
// int32 accumulators per 64 samples.
//
// Data path per 64-sample step:
//   global [t][i] bytes -> registers (one dword = 4 inputs of one sample)
//   -> 4x4 byte transposes (v_perm) -> [i][t] rows of 16 samples
//   -> CI4: nibble split by masking, giving 16*re and 16*im as exact int8
//      (the products then carry a factor 256, removed exactly at the end)
//   -> LDS (double buffered, rows padded to 80 bytes)
//   -> ds_read_b128 operand fragments -> MFMA.
// int32 partial sums are exact for at most 65535 samples (|16 x|^2 <= 2^15
// per sample and term pair); the host splits longer windows.
#include "xcorr_device.h"

namespace xcorr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kStep = 64;                  // samples per LDS stage
constexpr int kPitch = 80;                 // LDS bytes per row (64 samples + pad)
constexpr int kPart = kRowBlock * kPitch;  // one part (re or im) of a row block
constexpr int kSlotBytes = 2 * kPart;
constexpr int kBufBytes = kSlots * kSlotBytes;

// Per-thread staging job.  CI4: one wave stages one slot; thread q of the
// wave covers inputs 4*(q%16)..+3 and samples 16*(q/16)..+15 of the step.
// CI8: two jobs per thread, each an input pair and 16 samples.
template <int FMT>
struct Stager {
    static constexpr int kJobs = (FMT == 0) ? 1 : 2;
    uint32_t r[kJobs][16];
    __amdgpu_buffer_rsrc_t rsrc;  // this wave's channel; range = the chunk's samples
    uint32_t vofs[kJobs];         // byte offset of the job's column at sample 0
    int row[kJobs];               // first LDS row (input within the row block)
    int kofs[kJobs];              // byte offset of the 16-sample chunk in the row
    int row_bytes;
    int lds_slot;                 // slot index, -1 if the wave stages nothing

    __device__ __forceinline__ void init(const LaunchArgs& a, const WaveJob& w, int lane)
    {
        lds_slot = w.stage_rb < 0 ? -1 : w.wave;
        row_bytes = a.row_bytes;
        // Loads go through a buffer resource whose range ends at the chunk's
        // last sample, so samples past t_len (and whole channels past
        // n_channels, range 0) read as zero without a branch.
        rsrc = channel_rsrc(a, w.stage_rb, w.stage_ch);
#pragma unroll
        for (int j = 0; j < kJobs; ++j) {
            int col, tc;
            if (FMT == 0) { col = 4 * (lane & 15); tc = lane >> 4; }
            else          { col = 2 * (lane & 31); tc = (lane >> 5) + 2 * j; }
            row[j] = col;
            kofs[j] = 16 * tc;
            const int input = (w.stage_rb < 0 ? 0 : w.stage_rb) * kRowBlock + col;
            // a column past n_inputs gets an offset beyond every valid range
            vofs[j] = (uint32_t)(16 * tc) * (uint32_t)a.row_bytes +
                      column_offset(input, a.n_inputs, FMT == 0 ? 1 : 2);
        }
    }

    __device__ __forceinline__ void load(int t0)
    {
        const uint32_t step = (uint32_t)t0 * (uint32_t)row_bytes;
#pragma unroll
        for (int j = 0; j < kJobs; ++j) {
#pragma unroll
            for (int s = 0; s < 16; ++s)
                r[j][s] = load_b32(rsrc, vofs[j] + step + (uint32_t)s * (uint32_t)row_bytes);
        }
    }

    __device__ __forceinline__ void store(uint8_t* buf) const
    {
        if (lds_slot < 0) return;
        uint8_t* slot = buf + lds_slot * kSlotBytes;
#pragma unroll
        for (int j = 0; j < kJobs; ++j) {
            uint32_t o[4][4];               // o[g][m]: samples 4g..4g+3 of byte column m
#pragma unroll
            for (int g = 0; g < 4; ++g) transpose4(&r[j][4 * g], o[g]);
            if (FMT == 0) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    v4i re, im;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        re[g] = (int)(o[g][m] & 0xF0F0F0F0u);          // 16 * real
                        im[g] = (int)((o[g][m] << 4) & 0xF0F0F0F0u);   // 16 * imag
                    }
                    *(v4i*)(slot + (row[j] + m) * kPitch + kofs[j]) = re;
                    *(v4i*)(slot + kPart + (row[j] + m) * kPitch + kofs[j]) = im;
                }
            } else {
                // byte columns: re(2p), im(2p), re(2p+1), im(2p+1)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    v4i v;
#pragma unroll
                    for (int g = 0; g < 4; ++g) v[g] = (int)o[g][m];
                    const int part = m & 1, r_ = row[j] + (m >> 1);
                    *(v4i*)(slot + part * kPart + r_ * kPitch + kofs[j]) = v;
                }
            }
        }
    }
};

__device__ __forceinline__ v4i frag(const uint8_t* part, int blk, int lane)
{
    return *(const v4i*)(part + (16 * blk + (lane & 15)) * kPitch + 16 * (lane >> 4));
}

template <int FMT, int KIND>
__device__ __forceinline__ void run_tile(const LaunchArgs& a, const WaveJob& w, int lane, uint8_t* lds)
{
    Stager<FMT> st;
    st.init(a, w, lane);
    const int nk = (a.t_len + kStep - 1) / kStep;

    v4i acc_re[4][4], acc_ab[4][4], acc_ba[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            acc_re[bi][bj] = v4i{0, 0, 0, 0};
            acc_ab[bi][bj] = v4i{0, 0, 0, 0};
            acc_ba[bi][bj] = v4i{0, 0, 0, 0};
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
            v4i ia[4], ib[4], ja[4], jb[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                ia[b] = frag(pI, b, lane);
                ib[b] = frag(pI + kPart, b, lane);
            }
            if (KIND == KIND_DIAG) {
#pragma unroll
                for (int b = 0; b < 4; ++b) { ja[b] = ia[b]; jb[b] = ib[b]; }
            } else {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (block_on(KIND, 3, b)) {
                        ja[b] = frag(pJ, b, lane);
                        jb[b] = frag(pJ + kPart, b, lane);
                    }
                }
            }
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) {
                    if (!block_on(KIND, bi, bj)) continue;
                    acc_re[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ia[bi], ja[bj], acc_re[bi][bj], 0, 0, 0);
                    acc_re[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ib[bi], jb[bj], acc_re[bi][bj], 0, 0, 0);
                    acc_ab[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ia[bi], jb[bj], acc_ab[bi][bj], 0, 0, 0);
                    acc_ba[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ib[bi], ja[bj], acc_ba[bi][bj], 0, 0, 0);
                }
        }
        if (k + 1 < nk) st.store(lds + ((k + 1) & 1) * kBufBytes);
        __syncthreads();
    }
    if (KIND == KIND_NONE) return;

    // Epilogue: 16x16 int32 result blocks hold column (lane % 16) and rows
    // 4 * (lane / 16) + r in register r.
    const int ch = w.tile_ch;
    if (ch >= a.n_channels) return;
    const int i0 = w.rb_i * kRowBlock, j0 = w.rb_j * kRowBlock;
    const int shift = (FMT == 0) ? 8 : 0;
    const int64_t nb = (int64_t)a.n_inputs * (a.n_inputs + 1) / 2;
    const int64_t* src = (const int64_t*)a.src;
    int64_t* dst = (int64_t*)a.dst;
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
                int64_t re = ((int64_t)acc_re[bi][bj][r]) >> shift;
                int64_t im = ((int64_t)acc_ba[bi][bj][r] - (int64_t)acc_ab[bi][bj][r]) >> shift;
                const int64_t idx = ((int64_t)ch * nb + (int64_t)i * (i + 1) / 2 + j) * 2;
                if (src) {
                    const longlong2 s = *(const longlong2*)(src + idx);
                    re += s.x;
                    im += s.y;
                }
                longlong2 o;
                o.x = re;
                o.y = im;
                *(longlong2*)(dst + idx) = o;
            }
        }
}

template <int FMT>
__global__ void __launch_bounds__(kThreads, 1) xcorr_i8_kernel(LaunchArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kBufBytes];
    const int b = work_item_index(blockIdx.x, a.n_blocks, a.xcd_map);
    if (b >= a.n_blocks) return;
    const WaveJob w = wave_job(a, b);
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

hipError_t launch_i8(const LaunchArgs& a, int fmt, hipStream_t s)
{
    const dim3 grid(launch_blocks(a.n_blocks, a.xcd_map)), block(kThreads);
    if (fmt == 0) hipLaunchKernelGGL(xcorr_i8_kernel<0>, grid, block, 0, s, a);
    else          hipLaunchKernelGGL(xcorr_i8_kernel<1>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace xcorr
