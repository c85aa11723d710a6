// Internal definitions shared by the host code and the HIP kernels of libxcorr.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xcorr {

// ---------------------------------------------------------------------------
// Work decomposition.
//
// The lower triangle of one channel's N_i x N_i visibility matrix is cut into
// 64 x 64 tiles.  A workgroup stages up to four 64-input "row blocks" of the
// channel in LDS per time step; each wavefront accumulates a part of one tile
// (the rows of one staged row block, I, against the columns of another, J)
// for the whole time window.  A tile is a 4 x 4 grid of 16 x 16 blocks; a
// wave's kind says which blocks it owns:
//   FULL    all 16 (off-diagonal tile)
//   DIAG    the 10 blocks with bj <= bi (diagonal tile, I == J)
//   HALF0/1 the 8 blocks of columns bj 0-1 / 2-3
//   DIAG_A  (0,0) (1,0) (1,1) (3,2) (3,3)  }  the diagonal tile in two
//   DIAG_B  (2,0) (2,1) (2,2) (3,0) (3,1)  }  balanced halves of 5 blocks
// The four-wave kernels (fp16, fp32) use FULL/DIAG/HALF tiles; the eight-wave
// int8 kernel uses at most 10 blocks per wave so that its int32 accumulators
// fit two waves per SIMD.
// ---------------------------------------------------------------------------
enum TileKind : int8_t {
    KIND_NONE = 0, KIND_FULL = 1, KIND_DIAG = 2, KIND_HALF0 = 3, KIND_HALF1 = 4,
    KIND_DIAG_A = 5, KIND_DIAG_B = 6
};

// Bit 4*bi + bj set <=> block (bi, bj) belongs to the kind.
__host__ __device__ constexpr uint32_t kind_mask(int kind)
{
    return kind == KIND_FULL    ? 0xFFFFu
         : kind == KIND_DIAG    ? 0xF731u
         : kind == KIND_HALF0   ? 0x3333u
         : kind == KIND_HALF1   ? 0xCCCCu
         : kind == KIND_DIAG_A  ? 0xC031u
         : kind == KIND_DIAG_B  ? 0x3700u
         : 0u;
}

constexpr int kSlots = 4;          // row blocks staged per workgroup
constexpr int kRowBlock = 64;      // inputs per row block (= tile edge)
constexpr int kMaxWaves = 8;

struct WorkItem {                  // one workgroup's job inside one channel group
    int16_t rb[kSlots];            // row block staged in each slot, -1 = unused
    int8_t ch[kSlots];             // channel offset of each slot within its group
    int8_t wi[kMaxWaves];          // per wave: slot holding the tile's rows (I)
    int8_t wj[kMaxWaves];          // per wave: slot holding the tile's columns (J)
    int8_t kind[kMaxWaves];        // per wave: TileKind
    int32_t pad[3];
};
static_assert(sizeof(WorkItem) == 48, "WorkItem layout");

// Arguments of one accumulation launch (one time chunk).
struct LaunchArgs {
    const uint8_t* in;             // sample (channel 0, first time of the chunk)
    int64_t chan_stride;           // bytes between channels of the input
    int32_t row_bytes;             // bytes of one time sample of all inputs
    int32_t n_inputs;
    int32_t t_len;                 // samples in this chunk (>= 1)
    int32_t n_channels;
    int32_t ch_group;              // channels per work-item group
    int32_t n_items;               // work items per group
    int32_t n_blocks;              // total work items of the launch
    int32_t xcd_map;               // 1: XCD-aware block -> item mapping
    int32_t out32;                 // result mode: 0 int64 (re, im) pairs (src int64); 1 int32 pairs
                                   // (src int32); 2 int64 pairs added to an int32 src
    int32_t n_cols;                // inputs per row of the buffer read (>= n_inputs; the rest zero)
    const WorkItem* items;
    const void* src;               // optional accumulator to add (same layout as dst)
    void* dst;                     // result: [channel][tri][2]
    // null: the chunk's samples are rows 0 .. t_len - 1 from `in`.  Else
    // (persistent single-entry launches of the depth-4 LDS-DMA variants
    // only): sample k is row rows[k] from `in`, chan_stride bytes per
    // channel cover every row named, t_len <= kRowsCap of the format.
    const int32_t* rows;
};

// Most rows a launch with a row list takes (its LDS table: 32 KB beside the
// 4-bit variant's 64 KB of copy buffers, 16 KB beside the 8-bit one's 128 KB).
constexpr int kRowsCapCI4 = 8192;
constexpr int kRowsCapCI8 = 4096;

// Maps the hardware workgroup id to a work item.  Consecutive workgroup ids
// are dispatched round-robin over the 8 XCDs; giving each XCD a contiguous
// range of items keeps all workgroups of a channel on one XCD, so the
// channel's samples are fetched from HBM once and re-read from that XCD's L2.
__device__ inline int work_item_index(int block, int n_blocks, int xcd_map)
{
    if (!xcd_map) return block;
    const int per = (n_blocks + 7) >> 3;
    return (block & 7) * per + (block >> 3);
}

// One wave's share of a work item, read once into scalar registers.  With
// WAVES waves per workgroup, slot s is staged by waves s * WAVES/4 ...
template <int WAVES>
struct WaveJobT {
    int wave;                      // wave index in the workgroup
    int stage_part;                // which share of its slot this wave stages
    int stage_slot;                // slot this wave stages
    int stage_rb;                  // row block of that slot, -1 = none
    int stage_ch;                  // channel of that slot
    int kind;                      // TileKind of this wave's tile part
    int si, sj;                    // slots of the tile's rows and columns
    int rb_i, rb_j;                // row blocks of the tile's rows and columns
    int tile_ch;                   // channel of the tile
};

template <int WAVES>
__device__ inline WaveJobT<WAVES> wave_job(const LaunchArgs& a, int b)
{
    constexpr int per_slot = WAVES / kSlots;
    const int group = b / a.n_items;
    const WorkItem* it = a.items + (b - group * a.n_items);
    WaveJobT<WAVES> w;
    w.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    w.stage_slot = w.wave / per_slot;
    w.stage_part = w.wave - w.stage_slot * per_slot;
    w.stage_rb = __builtin_amdgcn_readfirstlane(it->rb[w.stage_slot]);
    w.stage_ch = group * a.ch_group + __builtin_amdgcn_readfirstlane(it->ch[w.stage_slot]);
    w.kind = __builtin_amdgcn_readfirstlane(it->kind[w.wave]);
    w.si = __builtin_amdgcn_readfirstlane(it->wi[w.wave]);
    w.sj = __builtin_amdgcn_readfirstlane(it->wj[w.wave]);
    w.rb_i = __builtin_amdgcn_readfirstlane(it->rb[w.si]);
    w.rb_j = __builtin_amdgcn_readfirstlane(it->rb[w.sj]);
    w.tile_ch = group * a.ch_group + __builtin_amdgcn_readfirstlane(it->ch[w.si]);
    return w;
}
using WaveJob = WaveJobT<4>;

inline int launch_blocks(int n_blocks, int xcd_map)
{
    return xcd_map ? ((n_blocks + 7) >> 3) << 3 : n_blocks;
}

// Arguments of one persistent batch launch: the launch arguments of up to
// kMaxBatchEntries (plan, time chunk) entries, passed by value.
constexpr int kMaxBatchEntries = 24;
// Work-queue counters of a launch: one per XCD and one count of finished
// workgroups (allocated zero; a persistent launch leaves them zero).
constexpr int kCounterInts = 16;
struct BatchArgs {
    int32_t n_entries;
    int32_t n_blocks;              // total work items over all entries
    int32_t xcd_map;               // 1: per-XCD slices; 0: one list for all
    int32_t pad;
    int32_t first[kMaxBatchEntries + 1];   // first global item of each entry
    int32_t slice[9];              // XCD x takes items [slice[x], slice[x+1])
    int* counters;                 // kCounterInts device ints, zero when the launch starts
    LaunchArgs e[kMaxBatchEntries];
};

// Tile variants of the int8 kernel (xcorr_plan_desc.tile).
constexpr int kTileDefault = 0;    // LDS-DMA, depth 4, where the shape allows
constexpr int kTileDma8 = 1;       // LDS-DMA staging, 8 copies in flight
constexpr int kTileDma4 = 2;       // LDS-DMA staging, 4 copies in flight
constexpr int kTileRegs = 3;       // register staging (byte transposes + LDS writes)

// Waves per workgroup of each kernel (the host plans work items to match).
constexpr int kWavesI8 = 8;
constexpr int kWavesF16 = 4;
constexpr int kWavesF32 = 4;

// Kernel launchers (one per arithmetic path); return the launch error.
// persist_grid > 0: LDS-DMA variants run as a persistent launch of that many
// workgroups (a multiple of 8); 0: one workgroup per work item.
// counters: kCounterInts device ints, zero, that the persistent launch's work
// queue uses and leaves zero.
hipError_t launch_i8(const LaunchArgs& a, int fmt, int tile, int persist_grid, int* counters, hipStream_t s);
hipError_t launch_i8_batch(const BatchArgs& ba, int fmt, int tile, int grid, hipStream_t s);
hipError_t launch_f16(const LaunchArgs& a, int fmt, hipStream_t s);
hipError_t launch_f32(const LaunchArgs& a, int fmt, hipStream_t s);
hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// out = a64 + a32 over n_pairs (re, im) pairs: out and a64 int64, a32 int32;
// either source may be null (zero); out may equal a64.
hipError_t launch_add_i32(void* out, const void* a64, const void* a32, size_t n_pairs, hipStream_t s);
// out[c][t] (rows of out_row bytes, out_row % 4 == 0) = in row (c, idx ? idx[t]
// : t) of in_row bytes (channel c at in + c * in_chan_stride), zero padded;
// t < n_rows, out channels n_rows rows apart.
hipError_t launch_pad_rows(uint8_t* out, int out_row, const uint8_t* in, int in_row, int64_t in_chan_stride,
                           const int32_t* idx, int64_t n_rows, int n_channels, hipStream_t s);

}  // namespace xcorr
