// Host-side state shared by the plan API (xcorr_api.cpp), the batch API
// (xcorr_batch.cpp) and the server (xcorr_server.cpp).
#pragma once

#include "xcorr.h"
#include "xcorr_internal.h"

#include <vector>

struct xcorr_plan_s {
    xcorr_plan_desc d;
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n_b = 0;                // baselines per channel
    size_t out_bytes = 0;
    void* acc = nullptr;            // accumulator, same layout as a dump
    bool acc_valid = false;         // false: accumulator is logically zero
    // int64 plans of the int8 path: launches that add to the integration
    // add into this int32 accumulator ([channel][tri][2] int32) instead of
    // reading and writing the int64 one; it is folded into acc (int64)
    // before it would hold more than fold_bound samples, and a dump adds
    // the two.  The integration is acc (if valid) + acc32 (if valid).
    void* acc32 = nullptr;
    bool acc32_valid = false;       // false: acc32 is logically zero
    int64_t samples32 = 0;          // samples summed in acc32 since its last fold
    int64_t acc32_bound = 0;        // most samples acc32 holds exactly
    xcorr::WorkItem* d_items = nullptr;
    std::vector<xcorr::WorkItem> h_items;
    int n_items = 0;                // items per channel group
    int ch_group = 1;
    int n_groups = 0;
    // Inputs per row of what the kernels read: n_inputs, or more when the
    // caller's rows must be staged zero padded (alignment of the kernels'
    // loads, or the 16-input rows of the LDS-DMA kernels).
    int n_cols = 0;
    uint8_t* d_pad = nullptr;       // padded copy of a chunk (grows on use)
    size_t pad_bytes = 0;
    int xcd_map = 1;
    int out32 = 0;                  // int32 (re, im) output (XCORR_FLAG_OUT_I32)
    int tile = 0;                   // int8 tile variant in use
    int persist_grid = 0;           // persistent workgroups of the LDS-DMA variants, 0 = off
    int* d_counters = nullptr;      // 8 work counters for batched launches over this plan
    uint8_t* d_tile_sel = nullptr;  // tile selection of xcorr_dump_tiles (allocated on first use)
    void* d_gate_buf = nullptr;     // gated accumulation: packed samples of all gates (grows on use)
    size_t gate_buf_bytes = 0;
    int32_t* d_gate_idx = nullptr;  // ... and their source sample indices
    size_t gate_idx_bytes = 0;
    int64_t fold_bound = 0;
    int64_t samples = 0;            // samples since the last reset
    int64_t window_start = 0;       // absolute sample index of the current window
    int64_t total = 0;              // absolute samples accumulated
    int64_t n_dumps = 0;
};

namespace xcorr {

xcorr_status fail(xcorr_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
xcorr_status hip_fail(hipError_t e, const char* what);
bool plan_live(xcorr_plan_t p);
xcorr_status check_ptr(const void* ptr, const char* name);
int64_t row_bytes_of(const xcorr_plan_s* p);
// Bytes per row of what the kernels read (n_cols inputs).
int64_t staged_row_bytes(const xcorr_plan_s* p);
// The buffer a chunk's launch reads: in itself, or (n_cols > n_inputs) a
// zero-padded copy in the plan's pad buffer, enqueued on stream.  in: the
// caller's layout (rows of n_inputs, channel c at in + c * chan_stride).
xcorr_status stage_chunk(xcorr_plan_s* p, const uint8_t* in, int64_t chan_stride, int64_t t_len, hipStream_t stream,
                         const uint8_t** out, int64_t* out_stride);
// Grows one of a plan's staging buffers to at least `need` bytes (waits for
// stream and the plan's stream first: the old buffer may be in use).
xcorr_status grow_buffer(xcorr_plan_s* p, hipStream_t stream, void** buf, size_t* bytes, size_t need, const char* what);
// Launch arguments of one time chunk of a plan.
LaunchArgs chunk_args(const xcorr_plan_s* p, const uint8_t* in, int64_t chan_stride, int32_t t_len,
                      const void* src, void* dst, int mode);
// The accumulators' state while the launches of a call are planned.
struct AccState {
    bool acc_valid, acc32_valid;
    int64_t samples32;
};
AccState acc_state(const xcorr_plan_s* p);
void set_acc_state(xcorr_plan_s* p, const AccState& s);
// Where one time chunk of len samples goes: the source its launch adds
// (null: none), its destination and its result mode (LaunchArgs.out32).
// final_dst: the chunk is the last of a fused dump and writes the dump
// there.  fold: the int32 accumulator must first be folded into the int64
// one (fold_acc32 with fold_acc_valid).  Updates s as if the launch ran.
struct ChunkTarget {
    const void* src;
    void* dst;
    int mode;
    bool fold, fold_acc_valid;
};
ChunkTarget chunk_target(const xcorr_plan_s* p, AccState& s, int64_t len, void* final_dst);
// acc = (acc_valid ? acc : 0) + acc32, enqueued on stream.
hipError_t fold_acc32(const xcorr_plan_s* p, bool acc_valid, hipStream_t stream);
// Writes the plan's integration (both accumulators, per its state) to out.
hipError_t launch_dump_of(const xcorr_plan_s* p, void* out, hipStream_t stream);
// Marks the integration empty (a dump with reset).
void reset_acc(xcorr_plan_s* p);
void fill_info(const xcorr_plan_s* p, xcorr_dump_info* info);
// XCORR_ERR_ARG if adding n_time samples would take an int32-output plan's
// window past its fold bound.
xcorr_status check_window(const xcorr_plan_s* p, int64_t n_time);
// Most samples one launch may take (int32 partials, 32-bit buffer ranges).
int64_t fold_bound_of(const xcorr_plan_desc* d);
// Enqueues the launches that accumulate n_time samples of every channel
// (channel c's rows start at in + c * chan_stride), split at the fold bound.
// If final_dst is non-null the last launch writes its result there instead
// of into the accumulator.
// staged: in already has rows of n_cols inputs (no padding pass).
xcorr_status run_window_strided(xcorr_plan_s* p, const uint8_t* in, int64_t chan_stride, int64_t n_time,
                                void* final_dst, bool staged = false);
// Most samples one launch of this plan may take through a row list (0: the
// plan cannot take row lists: they need a persistent depth-4 LDS-DMA int8
// plan reading the caller's rows as they are, and channels of chan_bytes <
// 2^31 bytes).
int row_list_cap(const xcorr_plan_s* p, int64_t chan_bytes);
// Accumulates the n samples of every channel whose rows are listed in rows
// (device, int32 row indices into the rows from in, channel c's at in + c *
// chan_stride), in launches of at most row_list_cap samples.
xcorr_status run_window_rows(xcorr_plan_s* p, const uint8_t* in, int64_t chan_stride, const int32_t* rows,
                             int64_t n);
// Inputs per row the kernels of a plan with this descriptor read.
int cols_of(const xcorr_plan_desc* d);
// Relative cost of a work item (MFMA blocks its waves own).
int item_blocks(const WorkItem& it);
// Work items of a plan (xcorr_items.cpp) for W row blocks of 64 inputs:
// items per group of ch_group channels.
void plan_items(int path, int W, std::vector<WorkItem>& items, int& ch_group);
// One fused window (accumulate + dump with reset) for each plan, all in one
// persistent launch per time chunk.  The plans must share the format.
xcorr_status run_fused_windows(hipStream_t stream, int* d_counters, const xcorr_batch_config& cfg,
                               const std::vector<xcorr_plan_t>& plans, const std::vector<const void*>& d_in,
                               const std::vector<int64_t>& n_time, const std::vector<void*>& d_out,
                               std::vector<xcorr_dump_info>& info);

}  // namespace xcorr
