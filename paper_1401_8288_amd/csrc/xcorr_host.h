// Host-side state shared by the plan API (xcorr_api.cpp), the batch API
// (xcorr_batch.cpp) and the server (xcorr_server.cpp).
#pragma once

#include "xcorr.h"
#include "xcorr_internal.h"

#include <vector>

// Channel groups of an 8-bit LDS-DMA chunk: the plane split of group g + 1
// runs beside the kernel of group g.
constexpr int kPlaneGroups = 8;

struct xcorr_plan_s {
    xcorr_plan_desc d;
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n_b = 0;                // baselines per channel
    size_t out_bytes = 0;
    void* acc = nullptr;            // accumulator, same layout as a dump
    bool acc_valid = false;         // false: accumulator is logically zero
    xcorr::WorkItem* d_items = nullptr;
    std::vector<xcorr::WorkItem> h_items;
    int n_items = 0;                // items per channel group
    int ch_group = 1;
    int n_groups = 0;
    // Launches that add to an accumulator (src != null) use a second table:
    // one channel per item, since the paired diagonal items of 4-bit plans
    // make those launches slower.  Equal to the first when nothing is paired.
    xcorr::WorkItem* d_items_src = nullptr;   // inside the d_items allocation
    std::vector<xcorr::WorkItem> h_items_src;
    int n_items_src = 0;
    int ch_group_src = 1;
    int n_groups_src = 0;
    size_t n_items_stored = 0;      // items in the d_items allocation
    int xcd_map = 1;
    int out32 = 0;                  // int32 (re, im) output (XCORR_FLAG_OUT_I32)
    int tile = 0;                   // int8 tile variant in use
    int persist_grid = 0;           // persistent workgroups of the LDS-DMA variants, 0 = off
    int* d_counters = nullptr;      // 8 work counters for batched launches over this plan
    uint8_t* d_tile_sel = nullptr;  // tile selection of xcorr_dump_tiles (allocated on first use)
    uint8_t* d_planes = nullptr;    // 8-bit LDS-DMA launches: the chunk with rows split into re | im planes
    size_t planes_bytes = 0;        // (grows on use)
    hipStream_t side = nullptr;     // ... whose plane split runs here, a channel group ahead of the
    hipEvent_t side_ev[kPlaneGroups + 1] = {};  // kernel (created on first use)
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
// Launch arguments of one time chunk of a plan.
LaunchArgs chunk_args(const xcorr_plan_s* p, const uint8_t* in, int64_t chan_stride, int32_t t_len,
                      const void* src, void* dst);
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
xcorr_status run_window_strided(xcorr_plan_s* p, const uint8_t* in, int64_t chan_stride, int64_t n_time,
                                void* final_dst);
// Relative cost of a work item (MFMA blocks its waves own).
int item_blocks(const WorkItem& it);
// Work items of a plan (xcorr_items.cpp): items / ch_group for launches that
// write their result, items_src / cg_src for launches that add to an
// accumulator; W row blocks of 64 inputs.
void plan_items(int path, int tile, int fmt, int W, std::vector<WorkItem>& items, int& ch_group,
                std::vector<WorkItem>& items_src, int& cg_src);
// Items a plan's device table holds for those two lists.
size_t stored_items(const std::vector<WorkItem>& items, int cg, const std::vector<WorkItem>& items_src, int cg_src);
// One fused window (accumulate + dump with reset) for each plan, all in one
// persistent launch per time chunk.  The plans must share the format.
xcorr_status run_fused_windows(hipStream_t stream, int* d_counters, const xcorr_batch_config& cfg,
                               const std::vector<xcorr_plan_t>& plans, const std::vector<const void*>& d_in,
                               const std::vector<int64_t>& n_time, const std::vector<void*>& d_out,
                               std::vector<xcorr_dump_info>& info);

}  // namespace xcorr
