// One integration window without any device allocation: the entry point for
// callers that cannot allocate (code under stream capture, serving loops,
// harnesses that forbid hipMalloc).  It runs the same kernels as
// xcorr_accumulate_dump on a freshly reset int8 plan, with the plan's
// device-side state -- the work-queue counters of the persistent launch and
// the work-item table -- held in a file-scope device array instead of a
// plan allocation.
#include "xcorr_host.h"

#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace xcorr {
namespace {

// Layout of the array: the counters first (zeroed by a fill kernel at the
// start of every call), the work-item table after them.
constexpr size_t kNoallocCounterBytes = 256;
constexpr size_t kNoallocBytes = (size_t)4 << 20;
constexpr size_t kNoallocMaxItems = (kNoallocBytes - kNoallocCounterBytes) / sizeof(WorkItem);
static_assert(kNoallocCounterBytes >= kCounterInts * sizeof(int), "counter area");

__device__ __align__(256) uint8_t scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;

struct DeviceState {
    uint8_t* ptr = nullptr;        // device address of `scratch` on this device
    int n_cu = 0;
    bool gfx950 = false;
};

std::mutex g_noalloc_mu;
DeviceState g_dev[kMaxDevices];

// Work-item tables by row-block count, built once and kept for the process,
// so that the host memory a queued copy reads stays valid.
struct Table {
    std::vector<WorkItem> items;
    int ch_group = 1;
};
std::map<int, Table> g_tables;

// The device's state, set up on the first call with that device current:
// the array's device address (the array's name is a host-side stand-in)
// and the properties the launch needs.
xcorr_status device_state(int dev, DeviceState& out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(XCORR_ERR_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    DeviceState& s = g_dev[dev];
    if (!s.ptr) {
        hipDeviceProp_t prop;
        hipError_t e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        s.n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        s.gfx950 = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        s.ptr = (uint8_t*)ptr;
    }
    out = s;
    return XCORR_OK;
}

const Table& table_for(int W)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_tables.find(W);
    if (it == g_tables.end()) {
        Table t;
        plan_items(XCORR_PATH_I8_MFMA, W, t.items, t.ch_group);
        it = g_tables.emplace(W, std::move(t)).first;
    }
    return it->second;
}

}  // namespace
}  // namespace xcorr

using namespace xcorr;

extern "C" xcorr_status xcorr_correlate_noalloc(const xcorr_plan_desc* d, const void* d_in, int64_t n_time,
                                                void* d_out)
{
    if (!d) return fail(XCORR_ERR_ARG, "null descriptor");
    if (d->path != XCORR_PATH_I8_MFMA) return fail(XCORR_ERR_UNSUPPORTED, "the no-allocation entry point is int8 only");
    if (d->format != XCORR_CI4 && d->format != XCORR_CI8) return fail(XCORR_ERR_ARG, "unknown format %d", d->format);
    if (d->n_inputs < 1 || d->n_channels < 1) return fail(XCORR_ERR_ARG, "n_inputs and n_channels must be >= 1");
    if (d->n_inputs > 32768) return fail(XCORR_ERR_UNSUPPORTED, "n_inputs %d above 32768", d->n_inputs);
    const int align = d->format == XCORR_CI4 ? 4 : 2;
    if (d->n_inputs % align)
        return fail(XCORR_ERR_UNSUPPORTED, "n_inputs must be a multiple of %d for this format", align);
    if (d->flags & ~(XCORR_FLAG_NO_XCD_MAP | XCORR_FLAG_NO_PERSIST | XCORR_FLAG_OUT_I32))
        return fail(XCORR_ERR_ARG, "unknown flags 0x%x", d->flags);
    if (d->tile != kTileDefault) return fail(XCORR_ERR_UNSUPPORTED, "the no-allocation entry point takes the default tile");
    const int64_t bound = fold_bound_of(d);
    if (n_time < 1 || n_time > bound)
        return fail(XCORR_ERR_ARG, "n_time %lld outside [1, %lld]: one window of one launch",
                    (long long)n_time, (long long)bound);
    xcorr_status s = check_ptr(d_in, "d_in");
    if (s == XCORR_OK) s = check_ptr(d_out, "d_out");
    if (s != XCORR_OK) return s;

    const int W = (d->n_inputs + kRowBlock - 1) / kRowBlock;
    const Table& t = table_for(W);
    if (t.items.size() > kNoallocMaxItems)
        return fail(XCORR_ERR_UNSUPPORTED, "%zu work items exceed the %zu the scratch array holds",
                    t.items.size(), kNoallocMaxItems);
    const int64_t n_groups = ((int64_t)d->n_channels + t.ch_group - 1) / t.ch_group;
    if ((int64_t)t.items.size() * n_groups > ((int64_t)1 << 30))
        return fail(XCORR_ERR_UNSUPPORTED, "too many work items");

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    DeviceState ds;
    s = device_state(dev, ds);
    if (s != XCORR_OK) return s;
    if (!ds.gfx950) return fail(XCORR_ERR_UNSUPPORTED, "device %d is not gfx950", dev);

    int* counters = (int*)ds.ptr;
    WorkItem* items = (WorkItem*)(ds.ptr + kNoallocCounterBytes);
    const hipStream_t stream = (hipStream_t)d->stream;

    LaunchArgs a;
    a.in = (const uint8_t*)d_in;
    a.row_bytes = d->n_inputs * (d->format == XCORR_CI4 ? 1 : 2);
    a.chan_stride = (int64_t)a.row_bytes * n_time;
    a.n_inputs = d->n_inputs;
    a.t_len = (int32_t)n_time;
    a.n_channels = d->n_channels;
    a.ch_group = t.ch_group;
    a.n_items = (int32_t)t.items.size();
    a.n_blocks = (int32_t)(t.items.size() * n_groups);
    a.xcd_map = (d->flags & XCORR_FLAG_NO_XCD_MAP) ? 0 : 1;
    a.out32 = (d->flags & XCORR_FLAG_OUT_I32) ? 1 : 0;
    a.n_cols = d->n_inputs;
    a.items = items;
    a.src = nullptr;
    a.dst = d_out;
    a.rows = nullptr;

    const int grid = (d->flags & XCORR_FLAG_NO_PERSIST) ? 0 : (ds.n_cu + 7) / 8 * 8;
    e = launch_fill_zero(counters, kNoallocCounterBytes, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(items, t.items.data(), t.items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_i8(a, d->format, kTileDefault, grid, counters, stream);
    if (e != hipSuccess) return hip_fail(e, "no-allocation window");
    return XCORR_OK;
}
