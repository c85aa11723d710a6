// Internal definitions shared by the host code and the HIP kernels of libxcorr.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xcorr {

// ---------------------------------------------------------------------------
// Work decomposition.
//
// The lower triangle of one channel's N_i x N_i visibility matrix is cut into
// 64 x 64 "wave tiles" (one wavefront accumulates one tile for the whole time
// window).  A workgroup of four wavefronts stages up to four 64-input "row
// blocks" of the channel in LDS per 64-sample step; each wave reads the row
// block of its tile's rows (I) and of its columns (J).  A tile is computed as
// a 4 x 4 grid of 16 x 16 blocks; its kind says which blocks:
//   FULL  all 16 (off-diagonal tile)
//   DIAG  the 10 blocks with bj <= bi (tile on the diagonal, I == J)
//   HALF0 columns 0-31 (bj 0, 1) of an off-diagonal tile
//   HALF1 columns 32-63 (bj 2, 3)
// ---------------------------------------------------------------------------
enum TileKind : int8_t { KIND_NONE = 0, KIND_FULL = 1, KIND_DIAG = 2, KIND_HALF0 = 3, KIND_HALF1 = 4 };

constexpr int kWaves = 4;          // wavefronts per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kSlots = 4;          // row blocks staged per workgroup
constexpr int kRowBlock = 64;      // inputs per row block (= wave tile edge)

struct WorkItem {                  // one workgroup's job inside one channel group
    int16_t rb[kSlots];            // row block staged in each slot, -1 = unused
    int8_t ch[kSlots];             // channel offset of each slot within its group
    int8_t wi[kWaves];             // per wave: slot holding the tile's rows (I)
    int8_t wj[kWaves];             // per wave: slot holding the tile's columns (J)
    int8_t kind[kWaves];           // per wave: TileKind
    int32_t pad[2];
};
static_assert(sizeof(WorkItem) == 32, "WorkItem layout");

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
    const WorkItem* items;
    const void* src;               // optional accumulator to add (same layout as dst)
    void* dst;                     // result: [channel][tri][2]
};

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

// One wave's share of a work item, read once into scalar registers.
struct WaveJob {
    int wave;                      // wave index in the workgroup (slot it stages)
    int stage_rb;                  // row block this wave stages, -1 = none
    int stage_ch;                  // channel of the staged row block
    int kind;                      // TileKind of this wave's tile
    int si, sj;                    // slots of the tile's rows and columns
    int rb_i, rb_j;                // row blocks of the tile's rows and columns
    int tile_ch;                   // channel of the tile
};

__device__ inline WaveJob wave_job(const LaunchArgs& a, int b)
{
    const int group = b / a.n_items;
    const WorkItem* it = a.items + (b - group * a.n_items);
    WaveJob w;
    w.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    w.stage_rb = __builtin_amdgcn_readfirstlane(it->rb[w.wave]);
    w.stage_ch = group * a.ch_group + __builtin_amdgcn_readfirstlane(it->ch[w.wave]);
    w.kind = __builtin_amdgcn_readfirstlane(it->kind[w.wave]);
    w.si = __builtin_amdgcn_readfirstlane(it->wi[w.wave]);
    w.sj = __builtin_amdgcn_readfirstlane(it->wj[w.wave]);
    w.rb_i = __builtin_amdgcn_readfirstlane(it->rb[w.si]);
    w.rb_j = __builtin_amdgcn_readfirstlane(it->rb[w.sj]);
    w.tile_ch = group * a.ch_group + __builtin_amdgcn_readfirstlane(it->ch[w.si]);
    return w;
}

inline int launch_blocks(int n_blocks, int xcd_map)
{
    return xcd_map ? ((n_blocks + 7) >> 3) << 3 : n_blocks;
}

// Kernel launchers (one per arithmetic path); return the launch error.
hipError_t launch_i8(const LaunchArgs& a, int fmt, hipStream_t s);
hipError_t launch_f16(const LaunchArgs& a, int fmt, hipStream_t s);
hipError_t launch_f32(const LaunchArgs& a, int fmt, hipStream_t s);
hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace xcorr
