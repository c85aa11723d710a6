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

#include <type_traits>
#include <utility>

namespace xcorr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kWaves = kWavesI8;
constexpr int kThreads = 64 * kWaves;
constexpr int kStep = 64;                  // samples per LDS stage
constexpr int kPitch = 80;                 // LDS bytes per row (64 samples + 16 pad)

// Kernel variants.  V_CI4: 4-bit samples, staged transposed ([input][time]
// rows) by byte permutes in registers.  V_CI8: 8-bit samples, the same with
// separate re and im rows.  V_CI4_DMA*: 4-bit samples with n_inputs % 16 == 0,
// copied by the buffer unit straight from HBM into LDS in their natural
// [time][input] order and transposed by the LDS transpose read
// (ds_read_b64_tr_b8); no vector registers or LDS writes are spent on staging.
// The DMA variant comes in two copy-pipeline depths (LDS buffers in flight),
// 4 and 8; the plan's tile setting or the autotuner picks one.  V_CI8_DMA4:
// 8-bit samples in rows of a multiple of 16 inputs, copied as they are
// (interleaved re, im bytes) and transposed by the 16-bit LDS transpose
// read (ds_read_b64_tr_b16), which gives a lane one input's (re, im) pairs
// of 4 consecutive samples; two byte permutes per dword then separate the
// real and imaginary operands.
// V_CI4_DMA4L, V_CI8_DMA4L: the same as V_CI4_DMA4, V_CI8_DMA4 for launches
// with a row list (LaunchArgs.rows), whose copies read listed rows.
enum Variant { V_CI4 = 0, V_CI8 = 1, V_CI4_DMA4 = 2, V_CI4_DMA8 = 3, V_CI8_DMA4 = 4, V_CI4_DMA4L = 5, V_CI8_DMA4L = 6 };
__host__ __device__ constexpr bool is_listed(int v) { return v == V_CI4_DMA4L || v == V_CI8_DMA4L; }
// The variant whose layout and fragments a variant uses.
__host__ __device__ constexpr int base_of(int v)
{
    return v == V_CI4_DMA4L ? V_CI4_DMA4 : v == V_CI8_DMA4L ? V_CI8_DMA4 : v;
}
__host__ __device__ constexpr bool is_ci4(int v) { return base_of(v) != V_CI8 && base_of(v) != V_CI8_DMA4; }
__host__ __device__ constexpr bool is_dma(int v)
{
    return base_of(v) == V_CI4_DMA4 || base_of(v) == V_CI4_DMA8 || base_of(v) == V_CI8_DMA4;
}
__host__ __device__ constexpr int dma_depth(int v) { return v == V_CI4_DMA8 ? 8 : 4; }
// LDS-DMA copies one wave issues per step (1 KB each).
__host__ __device__ constexpr int dma_copies(int v) { return base_of(v) == V_CI8_DMA4 ? 4 : 2; }

// Register-staged variants: global loads run kPrefetch steps ahead of the
// step they feed: a channel's first reader waits for HBM, and the other
// workgroups of the channel, which run at the same time on the same XCD, wait
// for the same lines.
constexpr int kPrefetch = 4;
// CI8 stages twice the bytes per thread: three steps ahead keep its loads in
// registers without spilling.
template <int FMT>
constexpr int kRing = FMT == V_CI8 ? 3 : kPrefetch;
// V_CI4_DMA*: LDS buffers, one per step in flight; the copy of step k + depth
// is issued while step k runs.
template <int FMT>
__device__ __forceinline__ constexpr int ring_depth() { return kRing<FMT>; }
template <int FMT>
__device__ __forceinline__ constexpr int n_buffers() { return is_dma(FMT) ? dma_depth(FMT) : 3; }
// Steps per unrolled loop iteration.
template <int FMT>
__device__ __forceinline__ constexpr int group_steps() { return is_dma(FMT) ? dma_depth(FMT) : kRing<FMT>; }

// LDS geometry.  CI4: one part per slot, the raw bytes (re and im nibbles)
// of 64 samples x 64 inputs, rows of 64 bytes padded to kPitch.  CI8: two
// parts, re rows and im rows.  V_CI4_DMA*: unpadded 64-byte sample rows.
// V_CI8_DMA4: unpadded 128-byte sample rows (64 inputs x (re, im)).
template <int FMT>
struct Geo {
    static constexpr int kParts = FMT == V_CI8 ? 2 : 1;
    static constexpr int kRowPitch = base_of(FMT) == V_CI8_DMA4 ? 2 * kRowBlock : is_dma(FMT) ? kRowBlock : kPitch;
    static constexpr int kPart = kRowBlock * kRowPitch;
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
    static constexpr int kJobs = (FMT == V_CI4) ? 1 : 2;
    uint32_t r[kRing<FMT>][kJobs][8];  // ring: slot k % depth holds step k
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
            const int col = (FMT == V_CI4) ? 4 * grp : 2 * (2 * grp + j);
            row[j] = col;
            const int input = (w.stage_rb < 0 ? 0 : w.stage_rb) * kRowBlock + col;
            vofs[j] = (uint32_t)(8 * g) * (uint32_t)a.row_bytes +
                      column_offset(input, a.n_inputs, FMT == V_CI4 ? 1 : 2);
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
                if (FMT == V_CI4) {
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

// V_CI4_DMA* staging.  A slot holds 64 sample rows of 64 bytes; 16-byte chunk
// q of row r sits at position q ^ swz(r).  The swizzle spreads the rows that
// one transpose read touches over all LDS banks (bits 1 and 2 of the row
// separate the rows of one 16-lane group, bits 2 and 4 those of one 32-lane
// group).  One LDS-DMA instruction fills 1 KB: lane l writes 16 bytes at
// 16 * l, i.e. row l / 4, position l % 4, so it loads chunk (l % 4) ^ swz(row)
// of its row.  The two waves of a slot copy 32 rows each in two instructions.
__device__ __forceinline__ int swz(int row)
{
    return ((row >> 2) & 1) | ((((row >> 1) ^ (row >> 4)) & 1) << 1);
}

struct DmaStager {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t vofs[2];
    int lds_ofs;
    int row_bytes;

    // A wave whose slot is unused copies zeros (its range is empty) into that
    // slot, which no wave reads; every wave thus issues the same loads.
    __device__ __forceinline__ void init(const LaunchArgs& a, const WaveJobT<kWaves>& w, int lane)
    {
        row_bytes = a.row_bytes;
        rsrc = channel_rsrc(a, w.stage_rb, w.stage_ch);
        lds_ofs = w.stage_slot * Geo<V_CI4_DMA8>::kSlotBytes + 32 * w.stage_part * kRowBlock;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int row = 32 * w.stage_part + 16 * j + (lane >> 2);
            const int q = (lane & 3) ^ swz(row);
            const int input = (w.stage_rb < 0 ? 0 : w.stage_rb) * kRowBlock + 16 * q;
            vofs[j] = (uint32_t)row * (uint32_t)a.row_bytes + column_offset(input, a.n_inputs, 1);
        }
    }

    // Copies the samples of step k into LDS buffer buf (past the chunk: zeros).
    __device__ __forceinline__ void load(uint8_t* buf, int k) const
    {
        typedef __attribute__((address_space(3))) void lds_void;
        const uint32_t step = (uint32_t)(k * kStep) * (uint32_t)row_bytes;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void*)(buf + lds_ofs + 16 * kRowBlock * j), 16,
                                                     (int)(vofs[j] + step), 0, 0, 0);
    }
};
template <>
struct Stager<V_CI4_DMA4> : DmaStager {};
template <>
struct Stager<V_CI4_DMA8> : DmaStager {};

// V_CI8_DMA4 staging.  A slot holds 64 sample rows of 128 bytes (64 inputs
// x (re, im)); 16-byte chunk q (8 inputs) of row r sits at position
// q ^ swz8(r).  A 16-bit transpose read takes, in each 16-lane group, 32
// bytes (two chunks) of 4 consecutive rows; two groups of one pass take rows
// 16 apart.  Rows of one parity in a pass then differ in bits 1 and 4, and
// mapping those bits to the XOR mask's bits 1 and 2 puts the pass's chunk
// pairs on distinct banks.  The mask does not depend on bits 2 and 3, so the
// four reads of a fragment (rows 4 apart) share one address.  One LDS-DMA
// instruction fills 1 KB: lane l writes 16 bytes at 16 * l, i.e. row l / 8,
// position l % 8; the two waves of a slot copy 32 rows each in four.
__device__ __forceinline__ int swz8(int row)
{
    return (((row >> 1) & 1) << 1) | (((row >> 4) & 1) << 2);
}

struct DmaStagerI {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t vofs[4];
    int lds_ofs;
    int row_bytes;

    __device__ __forceinline__ void init(const LaunchArgs& a, const WaveJobT<kWaves>& w, int lane)
    {
        row_bytes = a.row_bytes;
        rsrc = channel_rsrc(a, w.stage_rb, w.stage_ch);
        lds_ofs = w.stage_slot * Geo<V_CI8_DMA4>::kSlotBytes + 32 * w.stage_part * 2 * kRowBlock;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 32 * w.stage_part + 8 * j + (lane >> 3);
            const int q = (lane & 7) ^ swz8(row);
            const int input = (w.stage_rb < 0 ? 0 : w.stage_rb) * kRowBlock + 8 * q;
            vofs[j] = (uint32_t)row * (uint32_t)a.row_bytes + column_offset(input, a.n_inputs, 2);
        }
    }

    // Copies the samples of step k into LDS buffer buf (past the chunk: zeros).
    __device__ __forceinline__ void load(uint8_t* buf, int k) const
    {
        typedef __attribute__((address_space(3))) void lds_void;
        const uint32_t step = (uint32_t)(k * kStep) * (uint32_t)row_bytes;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void*)(buf + lds_ofs + 8 * 2 * kRowBlock * j), 16,
                                                     (int)(vofs[j] + step), 0, 0, 0);
    }
};
template <>
struct Stager<V_CI8_DMA4> : DmaStagerI {};

// Row lists (LaunchArgs.rows, the listed variants): the workgroup copies the
// chunk's list into an LDS table when the launch starts, and the copies of
// step k read row rows[64 k + r] of the window for the step's row r.  The
// channel's buffer range is all of its rows (chan_stride bytes).
template <int FMT>
__device__ __forceinline__ int32_t* lds_rows()
{
    static_assert(is_listed(FMT), "row tables of the listed variants");
    __shared__ int32_t tbl[base_of(FMT) == V_CI8_DMA4 ? kRowsCapCI8 : kRowsCapCI4];
    return tbl;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t listed_rsrc(const LaunchArgs& a, int rb, int ch)
{
    const bool ok = rb >= 0 && ch < a.n_channels;
    const uint8_t* base = a.in + (ok ? (int64_t)ch * a.chan_stride : 0);
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, ok ? (int)a.chan_stride : 0, kRsrcConfig);
}

// The copy stagers above with the step's rows looked up in the table: S is
// the base stager, R the rows one LDS-DMA instruction spans per lane group
// (16 for 64-byte rows, 8 for 128-byte rows).
template <int FMT, class S, int R>
struct ListedStager : S {
    const int32_t* tbl;
    int t_len;
    int row0;                      // this lane's first row of a step

    __device__ __forceinline__ void init(const LaunchArgs& a, const WaveJobT<kWaves>& w, int lane)
    {
        S::init(a, w, lane);
        this->rsrc = listed_rsrc(a, w.stage_rb, w.stage_ch);
        tbl = lds_rows<FMT>();
        t_len = a.t_len;
        row0 = 32 * w.stage_part + lane / (64 / R);
        // the base stager's offsets hold row * row_bytes + column: keep the columns
#pragma unroll
        for (int j = 0; j < (int)(sizeof(S::vofs) / sizeof(uint32_t)); ++j) {
            const uint32_t o = this->vofs[j];
            this->vofs[j] = o >= 0x80000000u ? 0x80000000u : o - (uint32_t)(row0 + R * j) * (uint32_t)a.row_bytes;
        }
    }

    __device__ __forceinline__ void load(uint8_t* buf, int k) const
    {
        typedef __attribute__((address_space(3))) void lds_void;
        constexpr int n = sizeof(S::vofs) / sizeof(uint32_t);
#pragma unroll
        for (int j = 0; j < n; ++j) {
            const int smp = k * kStep + row0 + R * j;
            const uint32_t col = this->vofs[j];
            const uint32_t ofs = (smp >= t_len || col == 0x80000000u)
                                     ? 0x80000000u
                                     : (uint32_t)tbl[smp] * (uint32_t)this->row_bytes + col;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(this->rsrc, (lds_void*)(buf + this->lds_ofs + 64 * R * (n == 2 ? 1 : 2) * j),
                                                     16, (int)ofs, 0, 0, 0);
        }
    }
};
template <>
struct Stager<V_CI4_DMA4L> : ListedStager<V_CI4_DMA4L, DmaStager, 16> {};
template <>
struct Stager<V_CI8_DMA4L> : ListedStager<V_CI8_DMA4L, DmaStagerI, 8> {};

// Offset of lane's first transpose read of block blk (16 inputs) of a
// V_CI8_DMA4 slot: the 16-lane group g takes samples 16 g..16 g + 15 in
// four reads of 4 rows (rows 16 g + 4 r + j / 4); lane j points at 8 bytes,
// quarter j % 4 of the block's 32 bytes, of its row.
__device__ __forceinline__ int tr16_offset(int slot, int blk, int lane)
{
    const int j = lane & 15;
    const int row = 16 * (lane >> 4) + (j >> 2);
    return slot * Geo<V_CI8_DMA4>::kSlotBytes + row * 2 * kRowBlock + 16 * ((2 * blk + ((j >> 1) & 1)) ^ swz8(row)) +
           8 * (j & 1);
}

// The raw words of one V_CI8_DMA4 fragment: lane l gets input l % 16's
// (re, im) pairs of 16 samples from four transpose reads (4 rows each, 512
// bytes apart); d[0] holds samples 0-7, d[1] samples 8-15.
__device__ __forceinline__ void frag_tr16(const uint8_t* buf, int ofs, v4i (&d)[2])
{
    typedef short v4s __attribute__((ext_vector_type(4)));
    typedef int v2i __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) v4s lds_v4s;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const v2i w = __builtin_bit_cast(
            v2i, __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(buf + ofs + 4 * r * 2 * kRowBlock)));
        d[r >> 1][2 * (r & 1)] = w.x;
        d[r >> 1][2 * (r & 1) + 1] = w.y;
    }
}

// Byte permutes that gather the even (re) and odd (im) bytes of a raw
// V_CI8_DMA4 fragment into the two MFMA operands.
__device__ __forceinline__ void split_tr16(const v4i (&d)[2], v4i& re, v4i& im)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t lo = (uint32_t)d[k >> 1][2 * (k & 1)], hi = (uint32_t)d[k >> 1][2 * (k & 1) + 1];
        re[k] = (int)__builtin_amdgcn_perm(hi, lo, 0x06040200u);
        im[k] = (int)__builtin_amdgcn_perm(hi, lo, 0x07050301u);
    }
}

// Operand fragment of a 16-row block: lane l holds row l % 16 and the 16
// samples 16 * (l / 16)..+15 of the step (the same sample set for the A and
// B operands of the MFMA, so the contraction pairs equal samples).
__device__ __forceinline__ v4i frag(const uint8_t* part, int blk, int lane)
{
    return *(const v4i*)(part + (16 * blk + (lane & 15)) * kPitch + 16 * (lane >> 4));
}

// The same fragment from a V_CI4_DMA* slot ([sample][input] rows): within
// each group of 16 lanes, lane j points at 8 bytes (inputs 8*(j%2)..+7 of the
// block) of sample row j/2, and the transpose read returns to lane L the
// byte of input L from each of the 8 rows.  Two reads give the 16 samples.
// ofs is the lane's byte offset of the block within the buffer (tr_offset).
__device__ __forceinline__ v4i frag_tr(const uint8_t* buf, int ofs)
{
    typedef int v2i __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) v2i lds_v2i;
    const v2i lo = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i*)(buf + ofs));
    const v2i hi = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i*)(buf + ofs + 8 * kRowBlock));
    return v4i{lo.x, lo.y, hi.x, hi.y};
}

__device__ __forceinline__ int tr_offset(int slot, int blk, int lane)
{
    const int j = lane & 15;
    const int row = 16 * (lane >> 4) + (j >> 1);
    return slot * Geo<V_CI4_DMA8>::kSlotBytes + row * kRowBlock + 16 * (blk ^ swz(row)) + 8 * (j & 1);
}

// Per-lane fragment offsets of the I and J slots (LDS-DMA variants).
struct FragOfs {
    int i[4], j[4];
};

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

// MFMA operands of one step: re and im fragments of the I and J row blocks
// (only the blocks the kind uses are set).
struct Ops {
    v4i ia[4], ib[4], ja[4], jb[4];
};

// Fragments as read from LDS.  CI4: raw bytes of the I and J blocks, split
// into operands by prepare().  CI8: the operands themselves.
template <int FMT>
struct Raw;
template <>
struct Raw<V_CI4> {
    v4i ri[4], rj[4];
};
template <>
struct Raw<V_CI4_DMA4> {
    v4i ri[4], rj[4];
};
template <>
struct Raw<V_CI4_DMA8> {
    v4i ri[4], rj[4];
};
template <>
struct Raw<V_CI8> {
    Ops o;
};
template <>
struct Raw<V_CI8_DMA4> {
    v4i ri[4][2], rj[4][2];
};
template <>
struct Raw<V_CI4_DMA4L> : Raw<V_CI4_DMA4> {};
template <>
struct Raw<V_CI8_DMA4L> : Raw<V_CI8_DMA4> {};

template <int KIND>
__device__ __forceinline__ constexpr bool same_block(int)
{
    return KIND == KIND_DIAG || KIND == KIND_DIAG_A || KIND == KIND_DIAG_B;
}

template <int KIND>
__device__ __forceinline__ constexpr bool need_i(int b)
{
    return row_on(KIND, b) || (same_block<KIND>(0) && column_on(KIND, b));
}

template <int KIND>
__device__ __forceinline__ constexpr bool need_j(int b)
{
    return column_on(KIND, b) && !same_block<KIND>(0);
}

template <int FMT, int KIND>
__device__ __forceinline__ void read_raw(const uint8_t* buf, int si, int sj, int lane, const FragOfs& fo,
                                         Raw<FMT>& r)
{
    const uint8_t* pI = buf + si * Geo<FMT>::kSlotBytes;
    const uint8_t* pJ = buf + sj * Geo<FMT>::kSlotBytes;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if constexpr (FMT == V_CI4) {
            if (need_i<KIND>(b)) r.ri[b] = frag(pI, b, lane);
            if (need_j<KIND>(b)) r.rj[b] = frag(pJ, b, lane);
        } else if constexpr (base_of(FMT) == V_CI8_DMA4) {
            if (need_i<KIND>(b)) frag_tr16(buf, fo.i[b], r.ri[b]);
            if (need_j<KIND>(b)) frag_tr16(buf, fo.j[b], r.rj[b]);
        } else if constexpr (is_dma(FMT)) {
            if (need_i<KIND>(b)) r.ri[b] = frag_tr(buf, fo.i[b]);
            if (need_j<KIND>(b)) r.rj[b] = frag_tr(buf, fo.j[b]);
        } else {
            if (need_i<KIND>(b)) {
                r.o.ia[b] = frag(pI, b, lane);
                r.o.ib[b] = frag(pI + Geo<FMT>::kPart, b, lane);
            }
            if (need_j<KIND>(b)) {
                r.o.ja[b] = frag(pJ, b, lane);
                r.o.jb[b] = frag(pJ + Geo<FMT>::kPart, b, lane);
            }
        }
    }
}

template <int FMT, int KIND>
__device__ __forceinline__ void prepare(const Raw<FMT>& r, Ops& o)
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if constexpr (is_ci4(FMT)) {
            if (need_i<KIND>(b)) {
                o.ia[b] = hi16(r.ri[b]);
                o.ib[b] = lo16(r.ri[b]);
            }
            if (need_j<KIND>(b)) {
                o.ja[b] = hi16(r.rj[b]);
                o.jb[b] = lo16(r.rj[b]);
            }
        } else if constexpr (base_of(FMT) == V_CI8_DMA4) {
            if (need_i<KIND>(b)) split_tr16(r.ri[b], o.ia[b], o.ib[b]);
            if (need_j<KIND>(b)) split_tr16(r.rj[b], o.ja[b], o.jb[b]);
        } else {
            if (need_i<KIND>(b)) { o.ia[b] = r.o.ia[b]; o.ib[b] = r.o.ib[b]; }
            if (need_j<KIND>(b)) { o.ja[b] = r.o.ja[b]; o.jb[b] = r.o.jb[b]; }
        }
        if constexpr (is_dma(FMT)) {
            // Keep the split in the step that read the fragments.  Without
            // these opaque copies the compiler folds the split of a group's
            // last step into the loop-carried value and redoes it at the top
            // of the next group, where it doubles that step's vector work
            // and holds back its first MFMAs (about 2 % of the launch).
            if (need_i<KIND>(b)) { asm("" : "+v"(o.ia[b])); asm("" : "+v"(o.ib[b])); }
            if (need_j<KIND>(b)) { asm("" : "+v"(o.ja[b])); asm("" : "+v"(o.jb[b])); }
        }
        if (same_block<KIND>(0) && column_on(KIND, b)) {
            o.ja[b] = o.ia[b];
            o.jb[b] = o.ib[b];
        }
    }
}

template <int KIND>
__device__ __forceinline__ constexpr int n_frags()
{
    int n = 0;
    for (int b = 0; b < 4; ++b) n += (need_i<KIND>(b) ? 1 : 0) + (need_j<KIND>(b) ? 1 : 0);
    return n;
}

// The block of a kind after block n (n = 4 * bi + bj), -1 after the last.
template <int KIND>
__device__ __forceinline__ constexpr int next_block(int n)
{
    for (int m = n + 1; m < 16; ++m)
        if (block_on(KIND, m >> 2, m & 3)) return m;
    return -1;
}

template <int KIND>
__device__ __forceinline__ constexpr int n_blocks()
{
    return __builtin_popcount(kind_mask(KIND));
}

// The MFMAs of one step, term-major so that the two MFMAs into one Re
// accumulator are far apart.
template <int KIND>
__device__ __forceinline__ void mma(const Ops& o, Acc& c)
{
#pragma unroll
    for (int term = 0; term < 4; ++term)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) {
                if (!block_on(KIND, bi, bj)) continue;
                if (term == 0) c.re[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ia[bi], o.ja[bj], c.re[bi][bj], 0, 0, 0);
                if (term == 1) c.ab[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ia[bi], o.jb[bj], c.ab[bi][bj], 0, 0, 0);
                if (term == 2) c.ba[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ib[bi], o.ja[bj], c.ba[bi][bj], 0, 0, 0);
                if (term == 3) c.re[bi][bj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ib[bi], o.jb[bj], c.re[bi][bj], 0, 0, 0);
            }
}

// LDS buffers of the pipeline.  V_CI4_DMA* gives every buffer its own LDS
// variable, so that the compiler can tell a copy into one buffer from the
// fragment reads of another and does not make those reads wait for it.
// The other variants index one array with a runtime step: p[0] is its base.
struct Bufs {
    uint8_t* p[8];
};

// Waits until at most N of this wave's vector-memory loads are in flight
// and all of its LDS reads have returned (expcnt left at its maximum).
template <int N>
__device__ __forceinline__ void wait_vm_lgkm()
{
    static_assert(N >= 0 && N < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | (0x7 << 4) | ((N >> 4) << 14));
}

// Workgroup barrier of the LDS-DMA pipeline.  A __syncthreads() fence would
// wait for every LDS-DMA copy in flight (they count as LDS writes); here the
// wave waits only for its copies older than the newest N and for its own
// LDS reads, which is all the next step needs.  The empty asm keeps the
// compiler from moving memory accesses across the barrier.
template <int N>
__device__ __forceinline__ void dma_barrier()
{
    __builtin_amdgcn_sched_barrier(0);
    wait_vm_lgkm<N>();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Issue pattern of one step: global loads, fragment reads, then the MFMAs
// each followed by a few vector instructions, then the LDS writes.
template <int FMT, int KIND>
__device__ __forceinline__ void schedule_step()
{
    constexpr int nm = 4 * n_blocks<KIND>();
    if constexpr (base_of(FMT) == V_CI8_DMA4) {
        // the four copies between the first MFMAs, then the fragment reads
        // after the next MFMAs, then the byte permutes after the rest
        constexpr int n_dsr = 4 * n_frags<KIND>();
        constexpr int n_valu = 8 * n_frags<KIND>();
        constexpr int a = nm / 16 > 0 ? nm / 16 : 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            __builtin_amdgcn_sched_group_barrier(0x008, a, 0);    // MFMA
            __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);    // VMEM (copy)
        }
        constexpr int rest = nm - 4 * a > 1 ? nm - 4 * a : 2;
        constexpr int rm = rest / 2;
        constexpr int rpm = (n_dsr + rm - 1) / rm;
        constexpr int vm = rest - rm;
        constexpr int vpm = (n_valu + vm - 1) / vm;
#pragma unroll
        for (int m = 0; m < rm; ++m) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, rpm, 0);  // DS read
        }
#pragma unroll
        for (int m = 0; m < vm; ++m) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, vpm, 0);  // VALU
        }
    } else if constexpr (is_dma(FMT)) {
        constexpr int n_dsr = 2 * n_frags<KIND>();
        constexpr int n_valu = 12 * n_frags<KIND>();
        // The copies and fragment reads are spread over the step so that no
        // wave stalls behind a burst of them: a few MFMAs, one copy, a few
        // MFMAs, the other copy, then one fragment read after each of the
        // next MFMAs, then the splitting work after each of the rest.
        constexpr int a = nm / 8 > 0 ? nm / 8 : 1;
        constexpr int rest = nm - 2 * a;
        constexpr int rm = (rest / 2 < n_dsr ? rest / 2 : n_dsr) > 0 ? (rest / 2 < n_dsr ? rest / 2 : n_dsr) : 1;
        constexpr int rpm = (n_dsr + rm - 1) / rm;
        constexpr int vm = rest - rm > 0 ? rest - rm : 1;
        constexpr int vpm = (n_valu + vm - 1) / vm;
        __builtin_amdgcn_sched_group_barrier(0x008, a, 0);        // MFMA
        __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);        // VMEM (copy)
        __builtin_amdgcn_sched_group_barrier(0x008, a, 0);
        __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
#pragma unroll
        for (int m = 0; m < rm; ++m) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, rpm, 0);  // DS read
        }
#pragma unroll
        for (int m = 0; m < vm; ++m) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, vpm, 0);  // VALU
        }
    } else {
        __builtin_amdgcn_sched_group_barrier(0x020, 8, 0);        // VMEM read
        __builtin_amdgcn_sched_group_barrier(0x100, n_frags<KIND>(), 0);   // DS read
#pragma unroll
        for (int m = 0; m < nm; ++m) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);    // VALU
        }
        __builtin_amdgcn_sched_group_barrier(0x200, 2, 0);        // DS write
    }
}

// V_CI4 and V_CI8: three LDS buffers, step k in buffer k % 3.  CI4 step k:
// load the samples of step k + D into ring slot S = k % D (D = 4; 3 for CI8),
// read the raw fragments of step k+1, run the MFMAs of step k from
// registers, split the step-k+1 fragments into operands, and write step k+2
// (ring slot (S+2) % D) into buffer (k+2) % 3.  The MFMAs are
// interleaved with the independent vector work of the next steps.  Buffer
// (k+2) % 3 last held step k-1, whose fragments were read in step k-2;
// buffer (k+1) % 3 was written in step k-1.  CI8 fragments are twice as
// large: they are read at the start of their own step from buffer k % 3.
//
// V_CI4_DMA*: D buffers (the depth), step k in buffer S = k % D.  Step k
// reads the fragments of step k+1, then refills buffer S (whose fragments,
// step k's, were read in step k-1) with step k + D, runs the MFMAs
// of step k and, before the barrier, waits for its own copy of step k+2: the
// copies of the D - 2 later steps may stay in flight.
template <int FMT, int KIND, int S>
__device__ __forceinline__ void pipeline_step(int k, Stager<FMT>& st, const Bufs& L, int si, int sj,
                                              int lane, const FragOfs& fo, Ops& ops, Acc& c)
{
    constexpr int B = Geo<FMT>::kBufBytes;
    uint8_t* lds = L.p[0];
    if constexpr (is_dma(FMT)) {
        constexpr int D = dma_depth(FMT);
        st.load(L.p[S], k + D);
        Ops nx;
        if constexpr (KIND != KIND_NONE) {
            Raw<FMT> raw;
            read_raw<FMT, KIND>(L.p[(S + 1) % D], si, sj, lane, fo, raw);
            mma<KIND>(ops, c);
            prepare<FMT, KIND>(raw, nx);
            schedule_step<FMT, KIND>();
        }
        dma_barrier<dma_copies(FMT) * (D - 2)>();
        ops = nx;
    } else if constexpr (is_ci4(FMT)) {
        constexpr int D = ring_depth<FMT>();
        uint8_t* next = lds + ((k + 1) % 3) * B;
        uint8_t* after = lds + ((k + 2) % 3) * B;
        st.template load<S % D>(k + D);
        Raw<FMT> raw;
        Ops nx;
        if (KIND != KIND_NONE) {
            read_raw<FMT, KIND>(next, si, sj, lane, fo, raw);
            mma<KIND>(ops, c);
            prepare<FMT, KIND>(raw, nx);
        }
        st.template store<(S + 2) % D>(after);
        if (KIND != KIND_NONE) schedule_step<FMT, KIND>();
        __syncthreads();
        ops = nx;
    } else {
        constexpr int D = ring_depth<FMT>();
        uint8_t* after = lds + ((k + 2) % 3) * B;
        st.template load<S % D>(k + D);
        if (KIND != KIND_NONE) {
            Raw<FMT> raw;
            read_raw<FMT, KIND>(lds + (k % 3) * B, si, sj, lane, fo, raw);
            prepare<FMT, KIND>(raw, ops);
            mma<KIND>(ops, c);
        }
        __builtin_amdgcn_sched_barrier(0);
        st.template store<(S + 2) % D>(after);
        __syncthreads();
    }
}

template <int FMT, int KIND, int... S>
__device__ __forceinline__ void pipeline_group(int k0, Stager<FMT>& st, const Bufs& L, int si, int sj,
                                               int lane, const FragOfs& fo, Ops& ops, Acc& c,
                                               std::integer_sequence<int, S...>)
{
    (pipeline_step<FMT, KIND, S>(k0 + S, st, L, si, sj, lane, fo, ops, c), ...);
}

// One work item.  st stages this item's samples.  After the item's steps
// (LDS-DMA variants) next(L) runs on every wave: a persistent workgroup
// learns its next item there and copies its first steps before this item's
// epilogue; the next item then starts with issue_prologue = false.
template <int FMT, int KIND, int O32, class Next>
__device__ __forceinline__ void run_tile(const LaunchArgs& a, const WaveJobT<kWaves>& w, int lane,
                                         const Bufs& L, Stager<FMT>& st, Next& next, bool issue_prologue)
{
    uint8_t* lds = L.p[0];
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
    FragOfs fo;
    if constexpr (is_dma(FMT)) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            fo.i[b] = base_of(FMT) == V_CI8_DMA4 ? tr16_offset(si, b, lane) : tr_offset(si, b, lane);
            fo.j[b] = base_of(FMT) == V_CI8_DMA4 ? tr16_offset(sj, b, lane) : tr_offset(sj, b, lane);
        }
    }

    // Prologue.  Loads past the window read zeros, and a step past it
    // multiplies zeros, so the steps run in unconditional groups; the
    // compiler can then count the loads in flight across the loop back-edge.
    constexpr int G = group_steps<FMT>();
    Ops ops;
    if constexpr (is_dma(FMT)) {
        // Copies of steps 0..D-1 into buffers 0..D-1 (unless the previous
        // item of a persistent workgroup issued them), operands of step 0;
        // the second barrier frees buffer 0 and publishes step 1.
        constexpr int D = dma_depth(FMT);
        if (issue_prologue) {
#pragma unroll
            for (int s = 0; s < D; ++s) st.load(L.p[s], s);
        }
        dma_barrier<dma_copies(FMT) * (D - 1)>();
        if (KIND != KIND_NONE) {
            Raw<FMT> raw;
            read_raw<FMT, KIND>(lds, si, sj, lane, fo, raw);
            prepare<FMT, KIND>(raw, ops);
        }
        dma_barrier<dma_copies(FMT) * (D - 2)>();
    } else {
        // Samples of steps 0..depth-1 into the ring, steps 0 and 1 into
        // LDS buffers 0 and 1, operands of step 0 (CI4).
        static_assert(kRing<FMT> == 3 || kRing<FMT> == 4, "ring of three or four slots");
        st.template load<0>(0);
        st.template load<1>(1);
        st.template load<2>(2);
        if constexpr (kRing<FMT> == 4) st.template load<3>(3);
        st.template store<0>(lds);
        st.template store<1>(lds + Geo<FMT>::kBufBytes);
        __syncthreads();
        if (is_ci4(FMT) && KIND != KIND_NONE) {
            Raw<FMT> raw;
            read_raw<FMT, KIND>(lds, si, sj, lane, fo, raw);
            prepare<FMT, KIND>(raw, ops);
        }
    }
    for (int k0 = 0; k0 < nk; k0 += G)
        pipeline_group<FMT, KIND>(k0, st, L, si, sj, lane, fo, ops, c, std::make_integer_sequence<int, G>());
    if constexpr (is_dma(FMT)) {
        // The copies issued by the last steps (zeros past the window) land
        // before the wave moves on.  Every wave passed the last barrier after
        // its last fragment reads, so a persistent workgroup can now copy its
        // next item's first steps, which then overlap this item's epilogue.
        wait_vm_lgkm<0>();
        next(L);
    }
    if (KIND == KIND_NONE) return;

    // Epilogue: 16x16 int32 result blocks hold column (lane % 16) and rows
    // 4 * (lane / 16) + r in register r.
    const int ch = w.tile_ch;
    if (ch >= a.n_channels) return;
    const int i0 = w.rb_i * kRowBlock, j0 = w.rb_j * kRowBlock;
    const int shift = is_ci4(FMT) ? 8 : 0;
    const int64_t nb = (int64_t)a.n_inputs * (a.n_inputs + 1) / 2;
    // Launches that add to a result (src, the plan's accumulator or the
    // previous chunk's output) read it here.  src may be dst, so the
    // compiler cannot move a load above an earlier store: in the LDS-DMA
    // variants an int32 source is loaded whole before the first store, and
    // an int64 one block by block ahead of the stores of the block before
    // it, so the wave waits for about one memory round trip per item (per
    // block in the register-staged variants, which have no registers to
    // spare) instead of one per row.
    // result mode OM: 0 int64 (re, im) adding int64, 1 int32 adding int32,
    // 2 int64 adding int32 (an int32 accumulator's last launch into a dump)
    typedef typename std::conditional<O32 == 1, int2, longlong2>::type Pair;
    typedef typename std::conditional<O32 == 0, longlong2, int2>::type SrcPair;
    const SrcPair* src = (const SrcPair*)a.src;
    Pair* dst = (Pair*)a.dst;
    const int jl = lane & 15, il = 4 * (lane >> 4);
    auto pair_index = [&](int n, int r, bool& ok) -> int64_t {
        const int i = i0 + 16 * (n >> 2) + il + r, j = j0 + 16 * (n & 3) + jl;
        ok = i < a.n_inputs && j <= i;
        return (int64_t)ch * nb + (int64_t)i * (i + 1) / 2 + j;
    };
    auto load_block = [&](int n, SrcPair (&v)[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bool ok;
            const int64_t q = pair_index(n, r, ok);
            v[r].x = 0;
            v[r].y = 0;
            if (ok) v[r] = src[q];
        }
    };
    if (!src) {
#pragma unroll
        for (int n = 0; n < 16; ++n) {
            if (!block_on(KIND, n >> 2, n & 3)) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                bool ok;
                const int64_t q = pair_index(n, r, ok);
                if (!ok) continue;
                Pair o;
                o.x = ((int64_t)c.re[n >> 2][n & 3][r]) >> shift;
                o.y = ((int64_t)c.ba[n >> 2][n & 3][r] - (int64_t)c.ab[n >> 2][n & 3][r]) >> shift;
                dst[q] = o;
            }
        }
        return;
    }
    if constexpr (O32 != 0 && is_dma(FMT)) {
        // int32 sources (2 registers a row): every block's source is loaded
        // before the first store, one memory round trip per item
        SrcPair all[16][4];
#pragma unroll
        for (int n = 0; n < 16; ++n)
            if (block_on(KIND, n >> 2, n & 3)) load_block(n, all[n]);
#pragma unroll
        for (int n = 0; n < 16; ++n) {
            if (!block_on(KIND, n >> 2, n & 3)) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                bool ok;
                const int64_t q = pair_index(n, r, ok);
                if (!ok) continue;
                Pair o;
                o.x = (((int64_t)c.re[n >> 2][n & 3][r]) >> shift) + (int64_t)all[n][r].x;
                o.y = (((int64_t)c.ba[n >> 2][n & 3][r] - (int64_t)c.ab[n >> 2][n & 3][r]) >> shift) +
                      (int64_t)all[n][r].y;
                dst[q] = o;
            }
        }
        return;
    }
    SrcPair cur[4], nxt[4];
    constexpr bool ahead = is_dma(FMT);
    if (ahead) load_block(next_block<KIND>(-1), nxt);
#pragma unroll
    for (int n = 0; n < 16; ++n) {
        if (!block_on(KIND, n >> 2, n & 3)) continue;
        if (ahead) {
#pragma unroll
            for (int r = 0; r < 4; ++r) cur[r] = nxt[r];
            if (next_block<KIND>(n) >= 0) load_block(next_block<KIND>(n), nxt);
        } else {
            load_block(n, cur);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bool ok;
            const int64_t q = pair_index(n, r, ok);
            if (!ok) continue;
            // int32 results are exact within the window bound the host enforces
            Pair o;
            o.x = (((int64_t)c.re[n >> 2][n & 3][r]) >> shift) + (int64_t)cur[r].x;
            o.y = (((int64_t)c.ba[n >> 2][n & 3][r] - (int64_t)c.ab[n >> 2][n & 3][r]) >> shift) + (int64_t)cur[r].y;
            dst[q] = o;
        }
    }
}

// The LDS buffers of a variant (kernel-lifetime LDS variables).
template <int FMT>
__device__ __forceinline__ Bufs lds_buffers()
{
    constexpr int B = Geo<FMT>::kBufBytes;
    Bufs L;
    if constexpr (is_dma(FMT)) {
        __shared__ __attribute__((aligned(16))) uint8_t b0[B], b1[B], b2[B], b3[B], b4[B], b5[B], b6[B], b7[B];
        uint8_t* const all[8] = {b0, b1, b2, b3, b4, b5, b6, b7};
#pragma unroll
        for (int i = 0; i < 8; ++i) L.p[i] = i < dma_depth(FMT) ? all[i] : nullptr;
    } else {
        __shared__ __attribute__((aligned(16))) uint8_t lds[3 * B];
#pragma unroll
        for (int i = 0; i < 8; ++i) L.p[i] = i < 3 ? lds + i * B : nullptr;
    }
    return L;
}

// One work item (local index b of the launch arguments a) by the whole
// workgroup.
template <int FMT, int O32, class Next>
__device__ __forceinline__ void dispatch_kind(const LaunchArgs& a, const WaveJobT<kWaves>& w, int lane,
                                              const Bufs& L, Stager<FMT>& st, Next& next, bool issue_prologue)
{
    switch (w.kind) {
    case KIND_HALF0:  run_tile<FMT, KIND_HALF0, O32>(a, w, lane, L, st, next, issue_prologue); break;
    case KIND_HALF1:  run_tile<FMT, KIND_HALF1, O32>(a, w, lane, L, st, next, issue_prologue); break;
    case KIND_DIAG_A: run_tile<FMT, KIND_DIAG_A, O32>(a, w, lane, L, st, next, issue_prologue); break;
    case KIND_DIAG_B: run_tile<FMT, KIND_DIAG_B, O32>(a, w, lane, L, st, next, issue_prologue); break;
    case KIND_DIAG:   run_tile<FMT, KIND_DIAG, O32>(a, w, lane, L, st, next, issue_prologue); break;
    default:          run_tile<FMT, KIND_NONE, O32>(a, w, lane, L, st, next, issue_prologue); break;
    }
}

// A workgroup that runs one item only.
struct NoNext {
    __device__ __forceinline__ void operator()(const Bufs&) {}
};

template <int FMT, int O32>
__device__ __forceinline__ void process_item(const LaunchArgs& a, int b, const Bufs& L)
{
    const WaveJobT<kWaves> w = wave_job<kWaves>(a, b);
    const int lane = threadIdx.x & 63;
    Stager<FMT> st;
    st.init(a, w, lane);
    NoNext none;
    dispatch_kind<FMT, O32>(a, w, lane, L, st, none, true);
}

__device__ __forceinline__ int entry_of(const BatchArgs& ba, int g)
{
    int e = 0;
    while (e + 1 < ba.n_entries && g >= ba.first[e + 1]) ++e;
    return e;
}

// One workgroup per work item of one plan's time chunk.
template <int FMT, int O32>
__global__ void __launch_bounds__(kThreads, 1) xcorr_i8_kernel(LaunchArgs a)
{
    const Bufs L = lds_buffers<FMT>();
    const int b = work_item_index(blockIdx.x, a.n_blocks, a.xcd_map);
    if (b >= a.n_blocks) return;
    process_item<FMT, O32>(a, b, L);
}

// The last workgroup to leave a launch that takes items from the per-XCD
// counters zeroes them for the next launch on the stream: every workgroup has taken its last claim before
// it counts itself out (counters[8]), so no claim follows the reset.
__device__ __forceinline__ void finish_queue(int* counters)
{
    if (threadIdx.x == 0 && atomicAdd(counters + 8, 1) == (int)gridDim.x - 1) {
#pragma unroll
        for (int q = 0; q <= 8; ++q) counters[q] = 0;
    }
}

// Persistent launch over the work items of several plans (subarrays of uneven
// size and window length).  The items of all entries form one list; XCD x
// owns the slice [slice[x], slice[x+1]) (contiguous, so a channel's workgroups
// share that XCD's L2) and its workgroups take items from it in order through
// the XCD's counter.  Every workgroup leaves once its slice is exhausted;
// the last one zeroes the counters.
template <int FMT, int O32>
__global__ void __launch_bounds__(kThreads, 1) xcorr_i8_batch_kernel(BatchArgs ba)
{
    const Bufs L = lds_buffers<FMT>();
    __shared__ int s_item;
    const int q = ba.xcd_map ? (int)(blockIdx.x & 7) : 0;
    const int lo = ba.xcd_map ? ba.slice[q] : ba.slice[0];
    const int hi = ba.xcd_map ? ba.slice[q + 1] : ba.slice[8];
    int* counter = ba.counters + q;
    for (;;) {
        if (threadIdx.x == 0) s_item = lo + atomicAdd(counter, 1);
        __syncthreads();
        const int g = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (g >= hi) break;
        const int e = entry_of(ba, g);
        process_item<FMT, O32>(ba.e[e], g - ba.first[e], L);
    }
    finish_queue(ba.counters);
}

// Persistent LDS-DMA kernel: the workgroups of XCD x take the items of
// slice [slice[x], slice[x+1]) from the XCD's counter (zero when the launch
// starts; the launch leaves it zero), one item ahead: a workgroup claims its next item when it starts
// the current one and reads the claim after the current item's steps, when
// every copy has landed, so the next item's first steps are still copied
// before the current epilogue.  A workgroup that starts late, or a CU that
// is busy with other work, then takes fewer items instead of holding up a
// fixed share of them.
template <int FMT>
struct PersistNext {
    const BatchArgs& ba;
    int* s_claim;                  // LDS slot that broadcasts the claim
    int claim;                     // thread 0: the counter value it claimed
    int lo, hi, lane;
    bool has;
    int g, e;
    WaveJobT<kWaves> w;
    Stager<FMT> st;

    __device__ __forceinline__ void operator()(const Bufs& L)
    {
        if (threadIdx.x == 0) *s_claim = lo + claim;
        dma_barrier<0>();
        g = __builtin_amdgcn_readfirstlane(*s_claim);
        has = g < hi;
        if (has) {
            e = entry_of(ba, g);
            w = wave_job<kWaves>(ba.e[e], g - ba.first[e]);
            st.init(ba.e[e], w, lane);
#pragma unroll
            for (int s = 0; s < dma_depth(FMT); ++s) st.load(L.p[s], s);
        }
    }
};

template <int FMT, int O32>
__global__ void __launch_bounds__(kThreads, 1) xcorr_i8_persist_kernel(BatchArgs ba)
{
    static_assert(is_dma(FMT), "persistent schedule of the LDS-DMA variants");
    const Bufs L = lds_buffers<FMT>();
    __shared__ int s_claim;
    const int q = ba.xcd_map ? (int)(blockIdx.x & 7) : 0;
    const int lo = ba.xcd_map ? ba.slice[q] : ba.slice[0];
    const int hi = ba.xcd_map ? ba.slice[q + 1] : ba.slice[8];
    int* counter = ba.counters + q;
    if (threadIdx.x == 0) s_claim = lo + atomicAdd(counter, 1);
    if constexpr (is_listed(FMT)) {
        // a row-list launch (one entry): its list into the LDS table
        int32_t* tbl = lds_rows<FMT>();
        for (int i = threadIdx.x; i < ba.e[0].t_len; i += kThreads) tbl[i] = ba.e[0].rows[i];
    }
    __syncthreads();
    int g = __builtin_amdgcn_readfirstlane(s_claim);
    if (g >= hi) {
        finish_queue(ba.counters);
        return;
    }
    const int lane = threadIdx.x & 63;
    int e = entry_of(ba, g);
    WaveJobT<kWaves> w = wave_job<kWaves>(ba.e[e], g - ba.first[e]);
    Stager<FMT> st;
    st.init(ba.e[e], w, lane);
    bool issue = true;
    for (;;) {
        PersistNext<FMT> next{ba, &s_claim, 0, lo, hi, lane, false, 0, 0, w, st};
        if (threadIdx.x == 0) next.claim = atomicAdd(counter, 1);
        dispatch_kind<FMT, O32>(ba.e[e], w, lane, L, st, next, issue);
        if (!next.has) break;
        g = next.g;
        e = next.e;
        w = next.w;
        st = next.st;
        issue = false;
    }
    finish_queue(ba.counters);
}

template <int FMT>
hipError_t launch_variant(const LaunchArgs& a, hipStream_t s)
{
    const dim3 grid(launch_blocks(a.n_blocks, a.xcd_map)), block(kThreads);
    if (a.out32 == 1)      hipLaunchKernelGGL((xcorr_i8_kernel<FMT, 1>), grid, block, 0, s, a);
    else if (a.out32 == 2) hipLaunchKernelGGL((xcorr_i8_kernel<FMT, 2>), grid, block, 0, s, a);
    else                   hipLaunchKernelGGL((xcorr_i8_kernel<FMT, 0>), grid, block, 0, s, a);
    return hipGetLastError();
}

// Every entry of a batched launch has the same result mode (the host splits
// mixed batches).
template <int FMT>
hipError_t launch_batch_variant(const BatchArgs& ba, int grid, hipStream_t s)
{
    const int om = ba.e[0].out32;
    const dim3 g(grid), b(kThreads);
    if constexpr (is_dma(FMT)) {
        if (om == 1)      hipLaunchKernelGGL((xcorr_i8_persist_kernel<FMT, 1>), g, b, 0, s, ba);
        else if (om == 2) hipLaunchKernelGGL((xcorr_i8_persist_kernel<FMT, 2>), g, b, 0, s, ba);
        else              hipLaunchKernelGGL((xcorr_i8_persist_kernel<FMT, 0>), g, b, 0, s, ba);
    } else {
        if (om == 1)      hipLaunchKernelGGL((xcorr_i8_batch_kernel<FMT, 1>), g, b, 0, s, ba);
        else if (om == 2) hipLaunchKernelGGL((xcorr_i8_batch_kernel<FMT, 2>), g, b, 0, s, ba);
        else              hipLaunchKernelGGL((xcorr_i8_batch_kernel<FMT, 0>), g, b, 0, s, ba);
    }
    return hipGetLastError();
}

// A single plan's chunk as a one-entry persistent launch (LDS-DMA variants).
template <int FMT>
hipError_t launch_persist_single(const LaunchArgs& a, int grid, int* counters, hipStream_t s)
{
    BatchArgs ba;
    __builtin_memset(&ba, 0, sizeof ba);
    ba.counters = counters;
    ba.n_entries = 1;
    ba.n_blocks = a.n_blocks;
    ba.xcd_map = a.xcd_map;
    ba.first[0] = 0;
    ba.first[1] = a.n_blocks;
    ba.e[0] = a;
    // equal slices rounded to whole channel groups
    const int per = (a.n_blocks / a.n_items + 7) / 8 * a.n_items;
    for (int x = 0; x <= 8; ++x) ba.slice[x] = x * per < a.n_blocks ? x * per : a.n_blocks;
    const int g = a.xcd_map ? grid : (a.n_blocks < grid ? a.n_blocks : grid);
    return launch_batch_variant<FMT>(ba, g, s);
}

// n_cols: inputs per row of the buffer the kernel reads.
int variant_of(int fmt, int n_cols, int tile)
{
    if (fmt == 1) return (tile == kTileRegs || n_cols % 16 != 0) ? V_CI8 : V_CI8_DMA4;
    if (tile == kTileRegs || n_cols % 16 != 0) return V_CI4;
    return tile == kTileDma8 ? V_CI4_DMA8 : V_CI4_DMA4;
}

}  // namespace

hipError_t launch_i8(const LaunchArgs& a, int fmt, int tile, int persist_grid, int* counters, hipStream_t s)
{
    if (a.rows) {
        // row lists: persistent launches of the depth-4 LDS-DMA variants
        const int v = variant_of(fmt, a.n_cols, tile);
        if (!persist_grid || (v != V_CI4_DMA4 && v != V_CI8_DMA4) ||
            a.t_len > (v == V_CI8_DMA4 ? kRowsCapCI8 : kRowsCapCI4) || a.chan_stride >= ((int64_t)1 << 31))
            return hipErrorInvalidValue;
        return v == V_CI4_DMA4 ? launch_persist_single<V_CI4_DMA4L>(a, persist_grid, counters, s)
                               : launch_persist_single<V_CI8_DMA4L>(a, persist_grid, counters, s);
    }
    switch (variant_of(fmt, a.n_cols, tile)) {
    case V_CI8:      return launch_variant<V_CI8>(a, s);
    case V_CI4:      return launch_variant<V_CI4>(a, s);
    case V_CI8_DMA4: return persist_grid ? launch_persist_single<V_CI8_DMA4>(a, persist_grid, counters, s)
                                         : launch_variant<V_CI8_DMA4>(a, s);
    case V_CI4_DMA4: return persist_grid ? launch_persist_single<V_CI4_DMA4>(a, persist_grid, counters, s)
                                         : launch_variant<V_CI4_DMA4>(a, s);
    default:         return persist_grid ? launch_persist_single<V_CI4_DMA8>(a, persist_grid, counters, s)
                                         : launch_variant<V_CI4_DMA8>(a, s);
    }
}

hipError_t launch_i8_batch(const BatchArgs& ba, int fmt, int tile, int grid, hipStream_t s)
{
    // one variant for the whole launch: the DMA variants need every entry's
    // n_inputs to be a multiple of 16
    int n16 = 1;
    for (int e = 0; e < ba.n_entries; ++e) n16 &= ba.e[e].n_cols % 16 == 0;
    switch (variant_of(fmt, n16 ? 16 : 4, tile)) {
    case V_CI8:      return launch_batch_variant<V_CI8>(ba, grid, s);
    case V_CI8_DMA4: return launch_batch_variant<V_CI8_DMA4>(ba, grid, s);
    case V_CI4:      return launch_batch_variant<V_CI4>(ba, grid, s);
    case V_CI4_DMA4: return launch_batch_variant<V_CI4_DMA4>(ba, grid, s);
    default:         return launch_batch_variant<V_CI4_DMA8>(ba, grid, s);
    }
}

}  // namespace xcorr
