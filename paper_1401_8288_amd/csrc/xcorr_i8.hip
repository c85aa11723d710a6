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
// Layout of the work: eight waves per workgroup, two per SIMD.  Each wave
// owns at most 8 of the 16 blocks of a 64x64 tile (96 int32 accumulator
// registers), so that the accumulators of both waves of a SIMD stay in
// VGPRs and the two waves fill each other's gaps in MFMA issue.
//
// Data path per 64-sample step:
//   global [t][i] bytes -> registers (one dword = 4 inputs of one sample)
//   -> 4x4 byte transposes (v_perm) -> [i][t] rows -> LDS (two buffers,
//      rows padded to 80 bytes); CI4 keeps the raw bytes, CI8 re and im rows
//   -> ds_read_b128 operand fragments
//   -> CI4: nibble split by masking, giving 16*re and 16*im as exact int8
//      (the products then carry a factor 256, removed exactly at the end)
//   -> MFMA.
// int32 partial sums are exact for at most 65535 samples (|16 x|^2 <= 2^15
// per sample and term pair); the host splits longer windows.
#include "xcorr_device.h"

namespace xcorr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kWaves = kWavesI8;
constexpr int kThreads = 64 * kWaves;
constexpr int kStep = 64;                  // samples per LDS stage
constexpr int kPitch = 80;                 // LDS bytes per row (64 samples + 16 pad)
// Global loads run this many steps ahead of the step they feed: a channel's
// first reader waits for HBM, and the other workgroups of the channel, which
// run at the same time on the same XCD, wait for the same lines.
constexpr int kPrefetch = 4;

// LDS geometry.  CI4: one part per slot, the raw transposed bytes (re and im
// nibbles of 64 samples per input row).  CI8: two parts, re rows and im rows.
template <int FMT>
struct Geo {
    static constexpr int kParts = FMT == 0 ? 1 : 2;
    static constexpr int kPart = kRowBlock * kPitch;
    static constexpr int kSlotBytes = kParts * kPart;
    static constexpr int kBufBytes = kSlots * kSlotBytes;
};

// Staging: the two waves of a slot share its 64 inputs x 64 samples.  Thread
// u (0..127 over the pair) takes the 8-sample chunk u % 8 and the input group
// u / 8: CI4 inputs 4*(u/8)..+3 (one job, 8 dword loads); CI8 input pairs
// 2*(2*(u/8) + j), j = 0, 1 (two jobs).  A group of 16 lanes of one
// ds_write_b64 covers two rows 4 apart (80 banks, 16 mod 32) and 64 bytes of
// each, i.e. all 32 banks once.
template <int FMT>
struct Stager {
    static constexpr int kJobs = (FMT == 0) ? 1 : 2;
    uint32_t r[kPrefetch][kJobs][8];  // ring: slot k % kPrefetch holds step k
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t vofs[kJobs];
    int row[kJobs];
    int kofs;
    int row_bytes;
    int lds_slot;

    __device__ __forceinline__ void init(const LaunchArgs& a, const WaveJobT<kWaves>& w, int lane)
    {
        lds_slot = w.stage_rb < 0 ? -1 : w.stage_slot;
        row_bytes = a.row_bytes;
        rsrc = channel_rsrc(a, w.stage_rb, w.stage_ch);
        const int u = 64 * w.stage_part + lane;
        const int g = u & 7, grp = u >> 3;
        kofs = 8 * g;
#pragma unroll
        for (int j = 0; j < kJobs; ++j) {
            const int col = (FMT == 0) ? 4 * grp : 2 * (2 * grp + j);
            row[j] = col;
            const int input = (w.stage_rb < 0 ? 0 : w.stage_rb) * kRowBlock + col;
            vofs[j] = (uint32_t)(8 * g) * (uint32_t)a.row_bytes +
                      column_offset(input, a.n_inputs, FMT == 0 ? 1 : 2);
        }
    }

    // Loads the samples of step k into ring slot S (reads past the chunk are zero).
    template <int S>
    __device__ __forceinline__ void load(int k)
    {
        const uint32_t step = (uint32_t)(k * kStep) * (uint32_t)row_bytes;
#pragma unroll
        for (int j = 0; j < kJobs; ++j)
#pragma unroll
            for (int s = 0; s < 8; ++s)
                r[S][j][s] = load_b32(rsrc, vofs[j] + step + (uint32_t)s * (uint32_t)row_bytes);
    }

    // Transposes ring slot S into the LDS buffer.
    template <int S>
    __device__ __forceinline__ void store(uint8_t* buf) const
    {
        if (lds_slot < 0) return;
        uint8_t* slot = buf + lds_slot * Geo<FMT>::kSlotBytes;
        typedef int v2i __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int j = 0; j < kJobs; ++j) {
            uint32_t o[2][4];               // o[G][m]: samples 4G..4G+3 of byte column m
            transpose4(&r[S][j][0], o[0]);
            transpose4(&r[S][j][4], o[1]);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const v2i v{(int)o[0][m], (int)o[1][m]};
                if (FMT == 0) {
                    *(v2i*)(slot + (row[j] + m) * kPitch + kofs) = v;
                } else {
                    // byte columns re(2p), im(2p), re(2p+1), im(2p+1)
                    const int part = m & 1, r_ = row[j] + (m >> 1);
                    *(v2i*)(slot + part * Geo<FMT>::kPart + r_ * kPitch + kofs) = v;
                }
            }
        }
    }
};

// Operand fragment of a 16-row block: lane l holds row l % 16 and the 16
// samples 16 * (l / 16)..+15 of the step (the same sample set for the A and
// B operands of the MFMA, so the contraction pairs equal samples).
__device__ __forceinline__ v4i frag(const uint8_t* part, int blk, int lane)
{
    return *(const v4i*)(part + (16 * blk + (lane & 15)) * kPitch + 16 * (lane >> 4));
}

// CI4 byte = (re << 4) | (im & 0xF): masking gives 16*re and 16*im as exact int8.
__device__ __forceinline__ v4i hi16(v4i x)
{
    const int m = (int)0xF0F0F0F0u;
    return x & v4i{m, m, m, m};
}
__device__ __forceinline__ v4i lo16(v4i x)
{
    const int m = (int)0xF0F0F0F0u;
    return (x << 4) & v4i{m, m, m, m};
}

struct Acc {
    v4i re[4][4], ab[4][4], ba[4][4];
};

// Reads the operands of the blocks the kind owns and runs its MFMAs.
template <int FMT, int KIND>
__device__ __forceinline__ void mfma_step(const uint8_t* buf, int si, int sj, int lane, Acc& c)
{
    const uint8_t* pI = buf + si * Geo<FMT>::kSlotBytes;
    const uint8_t* pJ = buf + sj * Geo<FMT>::kSlotBytes;
    v4i ia[4], ib[4], ja[4], jb[4];
    constexpr bool same = (KIND == KIND_DIAG || KIND == KIND_DIAG_A || KIND == KIND_DIAG_B);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (row_on(KIND, b) || (same && column_on(KIND, b))) {
            if (FMT == 0) {
                const v4i r = frag(pI, b, lane);
                ia[b] = hi16(r);
                ib[b] = lo16(r);
            } else {
                ia[b] = frag(pI, b, lane);
                ib[b] = frag(pI + Geo<FMT>::kPart, b, lane);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (!column_on(KIND, b)) continue;
        if (same) {
            ja[b] = ia[b];
            jb[b] = ib[b];
        } else if (FMT == 0) {
            const v4i r = frag(pJ, b, lane);
            ja[b] = hi16(r);
            jb[b] = lo16(r);
        } else {
            ja[b] = frag(pJ, b, lane);
            jb[b] = frag(pJ + Geo<FMT>::kPart, b, lane);
        }
    }
    // term-major order: the two MFMAs into one Re accumulator are far apart
#pragma unroll
    for (int term = 0; term < 4; ++term)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) {
                if (!block_on(KIND, bi, bj)) continue;
                if (term == 0) c.re[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ia[bi], ja[bj], c.re[bi][bj], 0, 0, 0);
                if (term == 1) c.ab[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ia[bi], jb[bj], c.ab[bi][bj], 0, 0, 0);
                if (term == 2) c.ba[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ib[bi], ja[bj], c.ba[bi][bj], 0, 0, 0);
                if (term == 3) c.re[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ib[bi], jb[bj], c.re[bi][bj], 0, 0, 0);
            }
}

// Step k, k % kPrefetch == S: load step k + kPrefetch into ring slot S, run
// the MFMAs of step k from LDS buffer k%2, write step k+1 from ring slot
// (S+1) % kPrefetch into buffer (k+1)%2.
template <int FMT, int KIND, int S>
__device__ __forceinline__ void pipeline_step(int k, Stager<FMT>& st, uint8_t* lds, int si, int sj,
                                              int lane, Acc& c)
{
    constexpr int B = Geo<FMT>::kBufBytes;
    st.template load<S>(k + kPrefetch);
    __builtin_amdgcn_sched_barrier(0);
    if (KIND != KIND_NONE) mfma_step<FMT, KIND>(lds + (k & 1) * B, si, sj, lane, c);
    __builtin_amdgcn_sched_barrier(0);
    st.template store<(S + 1) % kPrefetch>(lds + ((k + 1) & 1) * B);
    __syncthreads();
}

template <int FMT, int KIND>
__device__ __forceinline__ void run_tile(const LaunchArgs& a, const WaveJobT<kWaves>& w, int lane,
                                         uint8_t* lds)
{
    Stager<FMT> st;
    st.init(a, w, lane);
    const int nk = (a.t_len + kStep - 1) / kStep;

    Acc c;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            if (!block_on(KIND, bi, bj)) continue;
            c.re[bi][bj] = v4i{0, 0, 0, 0};
            c.ab[bi][bj] = v4i{0, 0, 0, 0};
            c.ba[bi][bj] = v4i{0, 0, 0, 0};
        }
    const int si = w.si, sj = w.sj;

    // Two LDS buffers: step k is read from buffer k%2 while the samples of
    // step k+1 (loaded kPrefetch steps earlier into ring slot (k+1) %
    // kPrefetch) are written to buffer (k+1)%2 at its end; the barrier that
    // closes step k-1 separates those writes from the last reads of buffer
    // (k+1)%2.  The loads of step k+kPrefetch go into the ring slot that held
    // step k.  Loads past the window read zeros and the stores they feed go
    // to a buffer no later step reads, so the steps need no branches.
#pragma unroll
    for (int s = 0; s < kPrefetch; ++s) {
        if (s == 0) st.template load<0>(0);
        if (s == 1) st.template load<1>(1);
        if (s == 2) st.template load<2>(2);
        if (s == 3) st.template load<3>(3);
    }
    st.template store<0>(lds);
    __syncthreads();
    // The steps run in groups of kPrefetch without conditions (a step past the
    // window multiplies zeros), so that the compiler can count the loads in
    // flight across the loop back-edge and wait only for the oldest group.
    static_assert(kPrefetch == 4, "the unrolled ring below assumes four slots");
    for (int k0 = 0; k0 < nk; k0 += kPrefetch) {
        pipeline_step<FMT, KIND, 0>(k0 + 0, st, lds, si, sj, lane, c);
        pipeline_step<FMT, KIND, 1>(k0 + 1, st, lds, si, sj, lane, c);
        pipeline_step<FMT, KIND, 2>(k0 + 2, st, lds, si, sj, lane, c);
        pipeline_step<FMT, KIND, 3>(k0 + 3, st, lds, si, sj, lane, c);
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
                int64_t re = ((int64_t)c.re[bi][bj][r]) >> shift;
                int64_t im = ((int64_t)c.ba[bi][bj][r] - (int64_t)c.ab[bi][bj][r]) >> shift;
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
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * Geo<FMT>::kBufBytes];
    const int b = work_item_index(blockIdx.x, a.n_blocks, a.xcd_map);
    if (b >= a.n_blocks) return;
    const WaveJobT<kWaves> w = wave_job<kWaves>(a, b);
    const int lane = threadIdx.x & 63;
    switch (w.kind) {
    case KIND_HALF0:  run_tile<FMT, KIND_HALF0>(a, w, lane, lds); break;
    case KIND_HALF1:  run_tile<FMT, KIND_HALF1>(a, w, lane, lds); break;
    case KIND_DIAG_A: run_tile<FMT, KIND_DIAG_A>(a, w, lane, lds); break;
    case KIND_DIAG_B: run_tile<FMT, KIND_DIAG_B>(a, w, lane, lds); break;
    case KIND_QUART0: run_tile<FMT, KIND_QUART0>(a, w, lane, lds); break;
    case KIND_QUART1: run_tile<FMT, KIND_QUART1>(a, w, lane, lds); break;
    case KIND_QUART2: run_tile<FMT, KIND_QUART2>(a, w, lane, lds); break;
    case KIND_QUART3: run_tile<FMT, KIND_QUART3>(a, w, lane, lds); break;
    default:          run_tile<FMT, KIND_NONE>(a, w, lane, lds); break;
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
