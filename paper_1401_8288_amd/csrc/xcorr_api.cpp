// Host side of libxcorr: argument checking, plan state, work decomposition
// and the launch sequence of accumulate / dump.  See include/xcorr.h.
#include "xcorr_host.h"
#include "xcorr_clock.h"
#include "xcorr_ct.h"
#include "xcorr_fstage.h"
#include "xcorr_tiles.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

using namespace xcorr;

namespace {
thread_local std::string g_err;
std::mutex g_mu;
std::set<xcorr_plan_t> g_live;
}  // namespace

namespace xcorr {

xcorr_status fail(xcorr_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

xcorr_status hip_fail(hipError_t e, const char* what)
{
    return fail(XCORR_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool plan_live(xcorr_plan_t p)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return p != nullptr && g_live.count(p) != 0;
}

xcorr_status check_ptr(const void* ptr, const char* name)
{
    if (!ptr) return fail(XCORR_ERR_ARG, "%s is null", name);
    if ((uintptr_t)ptr % 16) return fail(XCORR_ERR_ARG, "%s is not 16-byte aligned", name);
    return XCORR_OK;
}

int64_t row_bytes_of(const xcorr_plan_s* p)
{
    return (int64_t)p->d.n_inputs * (p->d.format == XCORR_CI4 ? 1 : 2);
}

int64_t staged_row_bytes(const xcorr_plan_s* p)
{
    return (int64_t)p->n_cols * (p->d.format == XCORR_CI4 ? 1 : 2);
}

// Zero inputs add nothing, so any input count can be padded.  The kernels
// load rows in dwords (4 inputs of 4-bit samples, 2 of 8-bit ones); the
// LDS-DMA int8 kernels read 16-input chunks.  Rows of other widths are
// padded to those multiples by a copy of each chunk (one pass over the
// input).  For fewer than 160 inputs, where the window is bound by HBM
// rather than by the matrix cores, the default tile keeps such rows in the
// register-staged kernel instead of paying that pass for the LDS-DMA one.
int cols_of(const xcorr_plan_desc* d)
{
    const int n = d->n_inputs;
    const int align = d->format == XCORR_CI4 ? 4 : 2;
    int c = (n + align - 1) / align * align;
    const bool dma_tile = d->tile == kTileDma4 || d->tile == kTileDma8;
    if (d->path == XCORR_PATH_I8_MFMA && n % 16 && (dma_tile || (d->tile == kTileDefault && n >= 160)))
        c = (n + 15) / 16 * 16;
    return c;
}

xcorr_status grow_buffer(xcorr_plan_s* p, hipStream_t stream, void** buf, size_t* bytes, size_t need, const char* what)
{
    if (*bytes >= need) return XCORR_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess && stream != p->stream) e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) {
        if (*buf) (void)hipFree(*buf);
        *buf = nullptr;
        *bytes = 0;
        e = hipMalloc(buf, need);
        if (e == hipSuccess) *bytes = need;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(XCORR_ERR_NOMEM, "%s (%zu bytes): %s", what, need, hipGetErrorString(e));
    }
    return XCORR_OK;
}

xcorr_status stage_chunk(xcorr_plan_s* p, const uint8_t* in, int64_t chan_stride, int64_t t_len, hipStream_t stream,
                         const uint8_t** out, int64_t* out_stride)
{
    if (p->n_cols == p->d.n_inputs) {
        *out = in;
        *out_stride = chan_stride;
        return XCORR_OK;
    }
    const int64_t srow = staged_row_bytes(p);
    xcorr_status s = grow_buffer(p, stream, (void**)&p->d_pad, &p->pad_bytes,
                                 (size_t)srow * t_len * p->d.n_channels, "row padding");
    if (s != XCORR_OK) return s;
    hipError_t e = launch_pad_rows(p->d_pad, (int)srow, in, (int)row_bytes_of(p), chan_stride, nullptr, t_len,
                                   p->d.n_channels, stream);
    if (e != hipSuccess) return hip_fail(e, "row padding");
    *out = p->d_pad;
    *out_stride = srow * t_len;
    return XCORR_OK;
}

LaunchArgs chunk_args(const xcorr_plan_s* p, const uint8_t* in, int64_t chan_stride, int32_t t_len,
                      const void* src, void* dst, int mode)
{
    LaunchArgs a;
    a.in = in;
    a.chan_stride = chan_stride;
    a.row_bytes = (int32_t)staged_row_bytes(p);
    a.n_cols = p->n_cols;
    a.n_inputs = p->d.n_inputs;
    a.t_len = t_len;
    a.n_channels = p->d.n_channels;
    a.ch_group = p->ch_group;
    a.n_items = p->n_items;
    a.n_blocks = p->n_items * p->n_groups;
    a.xcd_map = p->xcd_map;
    a.out32 = mode;
    a.items = p->d_items;
    a.src = src;
    a.dst = dst;
    a.rows = nullptr;
    return a;
}

AccState acc_state(const xcorr_plan_s* p)
{
    return AccState{p->acc_valid, p->acc32_valid, p->samples32};
}

void set_acc_state(xcorr_plan_s* p, const AccState& s)
{
    p->acc_valid = s.acc_valid;
    p->acc32_valid = s.acc32_valid;
    p->samples32 = s.samples32;
}

void reset_acc(xcorr_plan_s* p)
{
    set_acc_state(p, AccState{false, false, 0});
}

ChunkTarget chunk_target(const xcorr_plan_s* p, AccState& s, int64_t len, void* final_dst)
{
    ChunkTarget t{nullptr, nullptr, p->out32, false, false};
    if (!p->acc32) {
        // fp paths and int32-output plans: the accumulator has the result's type
        t.src = s.acc_valid ? p->acc : nullptr;
        t.dst = final_dst ? final_dst : p->acc;
        if (!final_dst) s.acc_valid = true;
        return t;
    }
    if (final_dst) {
        t.dst = final_dst;
        if (s.acc_valid) {
            if (s.acc32_valid) {
                t.fold = true;
                t.fold_acc_valid = true;
                s.acc32_valid = false;
                s.samples32 = 0;
            }
            t.src = p->acc;
            t.mode = 0;
        } else if (s.acc32_valid) {
            t.src = p->acc32;
            t.mode = 2;
        } else {
            t.mode = 0;
        }
        return t;
    }
    if (s.acc32_valid && s.samples32 + len > p->acc32_bound) {
        t.fold = true;
        t.fold_acc_valid = s.acc_valid;
        s.acc_valid = true;
        s.acc32_valid = false;
        s.samples32 = 0;
    }
    t.src = s.acc32_valid ? p->acc32 : nullptr;
    t.dst = p->acc32;
    t.mode = 1;
    s.acc32_valid = true;
    s.samples32 += len;
    return t;
}

hipError_t fold_acc32(const xcorr_plan_s* p, bool acc_valid, hipStream_t stream)
{
    return launch_add_i32(p->acc, acc_valid ? p->acc : nullptr, p->acc32, (size_t)p->n_b * p->d.n_channels, stream);
}

hipError_t launch_dump_of(const xcorr_plan_s* p, void* out, hipStream_t stream)
{
    if (p->acc32 && p->acc32_valid)
        return launch_add_i32(out, p->acc_valid ? p->acc : nullptr, p->acc32, (size_t)p->n_b * p->d.n_channels,
                              stream);
    return p->acc_valid ? launch_copy(out, p->acc, p->out_bytes, stream) : launch_fill_zero(out, p->out_bytes, stream);
}

int64_t fold_bound_of(const xcorr_plan_desc* d)
{
    // int8 path: int32 partial sums are exact for 65535 samples; fp paths
    // accumulate in fp32 without a count limit.
    const int64_t b = d->path == XCORR_PATH_I8_MFMA ? 65535 : (int64_t)1 << 30;
    // one launch's samples of one channel must stay below 2^31 bytes (the
    // kernels address a channel through a 32-bit buffer range)
    const int64_t row = (int64_t)cols_of(d) * (d->format == XCORR_CI4 ? 1 : 2);
    return std::min<int64_t>(b, ((int64_t)1 << 31) / row - 1);
}

xcorr_status check_window(const xcorr_plan_s* p, int64_t n_time)
{
    if (p->out32 && p->samples + n_time > p->fold_bound)
        return fail(XCORR_ERR_ARG, "int32 output: window of %lld samples past the bound %lld",
                    (long long)(p->samples + n_time), (long long)p->fold_bound);
    return XCORR_OK;
}

void fill_info(const xcorr_plan_s* p, xcorr_dump_info* info)
{
    if (!info) return;
    info->samples_accumulated = p->samples;
    info->start_sample = p->window_start;
    info->n_dumps = p->n_dumps;
}

}  // namespace xcorr

namespace {

using namespace xcorr;

void release(void* ptr)
{
    if (ptr) (void)hipFree(ptr);
}

bool live(xcorr_plan_t p) { return plan_live(p); }

size_t elem_bytes(const xcorr_plan_desc* d)
{
    return d->path == XCORR_PATH_I8_MFMA && !(d->flags & XCORR_FLAG_OUT_I32) ? 8 : 4;
}

xcorr_status check_desc(const xcorr_plan_desc* d)
{
    if (!d) return fail(XCORR_ERR_ARG, "null descriptor");
    if (d->format != XCORR_CI4 && d->format != XCORR_CI8)
        return fail(XCORR_ERR_ARG, "unknown format %d", d->format);
    if (d->path != XCORR_PATH_I8_MFMA && d->path != XCORR_PATH_F16_MFMA && d->path != XCORR_PATH_F32)
        return fail(XCORR_ERR_ARG, "unknown path %d", d->path);
    if (d->n_inputs < 1 || d->n_channels < 1)
        return fail(XCORR_ERR_ARG, "n_inputs and n_channels must be >= 1");
    if (d->n_inputs > 32768)
        return fail(XCORR_ERR_UNSUPPORTED, "n_inputs %d above 32768", d->n_inputs);
    if (d->flags & ~(XCORR_FLAG_NO_XCD_MAP | XCORR_FLAG_NO_PERSIST | XCORR_FLAG_OUT_I32))
        return fail(XCORR_ERR_ARG, "unknown flags 0x%x", d->flags);
    if ((d->flags & XCORR_FLAG_OUT_I32) && d->path != XCORR_PATH_I8_MFMA)
        return fail(XCORR_ERR_UNSUPPORTED, "int32 output exists for the int8 path");
    if (d->tile < 0 || d->tile > kTileRegs) return fail(XCORR_ERR_ARG, "unknown tile variant %d", d->tile);
    if (d->tile != kTileDefault && d->path != XCORR_PATH_I8_MFMA)
        return fail(XCORR_ERR_UNSUPPORTED, "tile variants exist for the int8 path only");
    if (d->tile == kTileDma8 && d->format != XCORR_CI4)
        return fail(XCORR_ERR_UNSUPPORTED, "the DMA8 tile takes 4-bit samples");
    return XCORR_OK;
}

// int64 plans of the int8 path hold an int32 accumulator beside the int64 one.
bool has_acc32(const xcorr_plan_desc* d)
{
    return d->path == XCORR_PATH_I8_MFMA && !(d->flags & XCORR_FLAG_OUT_I32);
}

size_t plan_device_bytes(const xcorr_plan_desc* d, size_t n_items)
{
    const int64_t n_b = (int64_t)d->n_inputs * (d->n_inputs + 1) / 2;
    const size_t acc = (size_t)n_b * d->n_channels * 2 * elem_bytes(d);
    return acc + (has_acc32(d) ? acc / 2 : 0) + n_items * sizeof(WorkItem) + 256 + 32;
}

// in: rows of n_cols inputs (already staged).  rows: the chunk's row list
// (row_list_ok plans only), or null.
xcorr_status launch_chunk(xcorr_plan_t p, const uint8_t* in, int64_t chan_stride, int32_t t_len,
                          const void* src, void* dst, int mode, const int32_t* rows = nullptr)
{
    LaunchArgs a = chunk_args(p, in, chan_stride, t_len, src, dst, mode);
    a.rows = rows;
    hipError_t e;
    switch (p->d.path) {
    case XCORR_PATH_I8_MFMA:
        e = launch_i8(a, p->d.format, p->tile, p->persist_grid, p->d_counters, p->stream);
        break;
    case XCORR_PATH_F16_MFMA: e = launch_f16(a, p->d.format, p->stream); break;
    default: e = launch_f32(a, p->d.format, p->stream); break;
    }
    if (e != hipSuccess) return hip_fail(e, "X-stage kernel launch");
    return XCORR_OK;
}

xcorr_status run_window(xcorr_plan_t p, const void* d_in, int64_t n_time, void* final_dst)
{
    return run_window_strided(p, (const uint8_t*)d_in, row_bytes_of(p) * n_time, n_time, final_dst);
}

}  // namespace

int xcorr::row_list_cap(const xcorr_plan_s* p, int64_t chan_bytes)
{
    if (p->d.path != XCORR_PATH_I8_MFMA || p->n_cols != p->d.n_inputs || p->n_cols % 16 || !p->persist_grid ||
        p->tile == kTileRegs || p->tile == kTileDma8 || chan_bytes >= ((int64_t)1 << 31))
        return 0;
    return p->d.format == XCORR_CI4 ? kRowsCapCI4 : kRowsCapCI8;
}

xcorr_status xcorr::run_window_rows(xcorr_plan_t p, const uint8_t* in, int64_t chan_stride, const int32_t* rows,
                                    int64_t n)
{
    const int64_t cap = std::min<int64_t>(p->fold_bound, row_list_cap(p, chan_stride));
    if (cap <= 0) return fail(XCORR_ERR_UNSUPPORTED, "row lists need a persistent depth-4 LDS-DMA int8 plan");
    AccState st = acc_state(p);
    for (int64_t t0 = 0; t0 < n; t0 += cap) {
        const int64_t len = std::min<int64_t>(cap, n - t0);
        const ChunkTarget t = chunk_target(p, st, len, nullptr);
        if (t.fold) {
            hipError_t e = fold_acc32(p, t.fold_acc_valid, p->stream);
            if (e != hipSuccess) return hip_fail(e, "int32 accumulator fold");
        }
        xcorr_status s = launch_chunk(p, in, chan_stride, (int32_t)len, t.src, t.dst, t.mode, rows + t0);
        if (s != XCORR_OK) return s;
        set_acc_state(p, st);
    }
    return XCORR_OK;
}

xcorr_status xcorr::run_window_strided(xcorr_plan_t p, const uint8_t* in, int64_t chan_stride,
                                       int64_t n_time, void* final_dst, bool staged)
{
    const int64_t row = staged ? staged_row_bytes(p) : row_bytes_of(p);
    AccState st = acc_state(p);
    for (int64_t t0 = 0; t0 < n_time; t0 += p->fold_bound) {
        const int64_t len = std::min<int64_t>(p->fold_bound, n_time - t0);
        const bool last = t0 + len >= n_time;
        const ChunkTarget t = chunk_target(p, st, len, last ? final_dst : nullptr);
        if (t.fold) {
            hipError_t e = fold_acc32(p, t.fold_acc_valid, p->stream);
            if (e != hipSuccess) return hip_fail(e, "int32 accumulator fold");
        }
        const uint8_t* cin = in + t0 * row;
        int64_t cstride = chan_stride;
        if (!staged) {
            xcorr_status s = stage_chunk(p, cin, chan_stride, len, p->stream, &cin, &cstride);
            if (s != XCORR_OK) return s;
        }
        xcorr_status s = launch_chunk(p, cin, cstride, (int32_t)len, t.src, t.dst, t.mode);
        if (s != XCORR_OK) return s;
        set_acc_state(p, st);
    }
    return XCORR_OK;
}

extern "C" {

int32_t xcorr_version(void) { return 100; }

const char* xcorr_last_error(void) { return g_err.c_str(); }

const char* xcorr_strerror(xcorr_status s)
{
    switch (s) {
    case XCORR_OK: return "ok";
    case XCORR_ERR_ARG: return "invalid argument";
    case XCORR_ERR_NOMEM: return "out of device memory";
    case XCORR_ERR_DEVICE: return "device (HIP) error";
    case XCORR_ERR_STATE: return "invalid plan handle";
    case XCORR_ERR_UNSUPPORTED: return "unsupported device or shape";
    }
    return "unknown status";
}

xcorr_status xcorr_plan_bytes(const xcorr_plan_desc* d, size_t* bytes)
{
    xcorr_status s = check_desc(d);
    if (s != XCORR_OK) return s;
    if (!bytes) return fail(XCORR_ERR_ARG, "null output");
    std::vector<WorkItem> items;
    int cg;
    plan_items(d->path, (d->n_inputs + kRowBlock - 1) / kRowBlock, items, cg);
    *bytes = plan_device_bytes(d, items.size());
    return XCORR_OK;
}

xcorr_status xcorr_plan(xcorr_plan_t* out, const xcorr_plan_desc* d)
{
    if (!out) return fail(XCORR_ERR_ARG, "null plan output");
    xcorr_status s = check_desc(d);
    if (s != XCORR_OK) return s;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(XCORR_ERR_UNSUPPORTED, "device %d is %s, not gfx950", dev, prop.gcnArchName);

    xcorr_plan_t p = new (std::nothrow) xcorr_plan_s();
    if (!p) return fail(XCORR_ERR_NOMEM, "host allocation");
    p->d = *d;
    p->device = dev;
    p->stream = (hipStream_t)d->stream;
    p->n_b = (int64_t)d->n_inputs * (d->n_inputs + 1) / 2;
    p->out_bytes = (size_t)p->n_b * d->n_channels * 2 * elem_bytes(d);
    p->xcd_map = (d->flags & XCORR_FLAG_NO_XCD_MAP) ? 0 : 1;
    p->out32 = (d->flags & XCORR_FLAG_OUT_I32) ? 1 : 0;
    // LDS-DMA chunks run as a persistent launch of one workgroup per CU
    const int n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    p->persist_grid = (d->flags & XCORR_FLAG_NO_PERSIST) ? 0 : (n_cu + 7) / 8 * 8;
    p->fold_bound = fold_bound_of(d);
    p->n_cols = cols_of(d);
    // the int32 accumulator holds true sums (not the kernel's scaled
    // partials): at most 2 * 8 * 8 = 128 per sample for 4-bit samples and
    // 2 * 128 * 128 for 8-bit samples in magnitude
    p->acc32_bound = d->format == XCORR_CI4 ? 16777215 : 65535;

    p->tile = d->tile;
    std::vector<WorkItem>& items = p->h_items;
    plan_items(d->path, (d->n_inputs + kRowBlock - 1) / kRowBlock, items, p->ch_group);
    p->n_items = (int)items.size();
    p->n_groups = (d->n_channels + p->ch_group - 1) / p->ch_group;
    const int64_t blocks = (int64_t)p->n_items * p->n_groups;
    if (blocks > (int64_t)1 << 30) {
        delete p;
        return fail(XCORR_ERR_UNSUPPORTED, "too many work items");
    }

    e = hipMalloc(&p->acc, p->out_bytes);
    if (e == hipSuccess && has_acc32(d)) e = hipMalloc(&p->acc32, p->out_bytes / 2);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_items, items.size() * sizeof(WorkItem));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_counters, kCounterInts * sizeof(int));
    if (e == hipSuccess) e = hipMemset(p->d_counters, 0, kCounterInts * sizeof(int));
    if (e != hipSuccess) {
        release(p->acc);
        release(p->acc32);
        release(p->d_items);
        release(p->d_counters);
        delete p;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? XCORR_ERR_NOMEM : XCORR_ERR_DEVICE,
                    "plan allocation: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_items, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(p->acc);
        release(p->acc32);
        release(p->d_items);
        release(p->d_counters);
        delete p;
        return hip_fail(e, "work item upload");
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(p);
    }
    *out = p;
    return XCORR_OK;
}

xcorr_status xcorr_accumulate(xcorr_plan_t p, const void* d_in, int64_t n_time)
{
    if (!live(p)) return fail(XCORR_ERR_STATE, "invalid plan handle");
    if (n_time < 0) return fail(XCORR_ERR_ARG, "negative n_time");
    if (n_time == 0) return XCORR_OK;
    xcorr_status s = check_ptr(d_in, "d_in");
    if (s == XCORR_OK) s = check_window(p, n_time);
    if (s != XCORR_OK) return s;
    s = run_window(p, d_in, n_time, nullptr);
    if (s != XCORR_OK) return s;
    p->samples += n_time;
    p->total += n_time;
    return XCORR_OK;
}

xcorr_status xcorr_dump(xcorr_plan_t p, void* d_out, int reset, xcorr_dump_info* info)
{
    if (!live(p)) return fail(XCORR_ERR_STATE, "invalid plan handle");
    xcorr_status s = check_ptr(d_out, "d_out");
    if (s != XCORR_OK) return s;
    hipError_t e = launch_dump_of(p, d_out, p->stream);
    if (e != hipSuccess) return hip_fail(e, "dump");
    p->n_dumps += 1;
    fill_info(p, info);
    if (reset) {
        reset_acc(p);
        p->samples = 0;
        p->window_start = p->total;
    }
    return XCORR_OK;
}

xcorr_status xcorr_accumulate_dump(xcorr_plan_t p, const void* d_in, int64_t n_time, void* d_out,
                                   int reset, xcorr_dump_info* info)
{
    if (!live(p)) return fail(XCORR_ERR_STATE, "invalid plan handle");
    if (n_time < 0) return fail(XCORR_ERR_ARG, "negative n_time");
    xcorr_status s = check_ptr(d_out, "d_out");
    if (s != XCORR_OK) return s;
    if (n_time == 0) return xcorr_dump(p, d_out, reset, info);
    s = check_ptr(d_in, "d_in");
    if (s == XCORR_OK) s = check_window(p, n_time);
    if (s != XCORR_OK) return s;
    if (reset) {
        // the last launch writes the dump directly; the accumulator restarts
        s = run_window(p, d_in, n_time, d_out);
        if (s != XCORR_OK) return s;
        reset_acc(p);
    } else {
        s = run_window(p, d_in, n_time, nullptr);
        if (s != XCORR_OK) return s;
        hipError_t e = launch_dump_of(p, d_out, p->stream);
        if (e != hipSuccess) return hip_fail(e, "dump copy");
    }
    p->samples += n_time;
    p->total += n_time;
    p->n_dumps += 1;
    fill_info(p, info);
    if (reset) {
        p->samples = 0;
        p->window_start = p->total;
    }
    return XCORR_OK;
}

xcorr_status xcorr_query(xcorr_plan_t p, xcorr_plan_info* info)
{
    if (!live(p)) return fail(XCORR_ERR_STATE, "invalid plan handle");
    if (!info) return fail(XCORR_ERR_ARG, "null info");
    info->device_bytes = plan_device_bytes(&p->d, p->h_items.size());
    info->output_bytes = p->out_bytes;
    info->input_bytes_per_sample =
        (size_t)p->d.n_inputs * (p->d.format == XCORR_CI4 ? 1 : 2) * p->d.n_channels;
    info->fold_bound = p->fold_bound;
    info->tile = p->tile;
    info->work_items = p->n_items * p->n_groups;
    info->items_per_group = p->n_items;
    info->channels_per_group = p->ch_group;
    return XCORR_OK;
}

xcorr_status xcorr_dump_tiles(xcorr_plan_t p, void* d_out, const uint8_t* tile_select, int reset,
                              xcorr_dump_info* info)
{
    if (!live(p)) return fail(XCORR_ERR_STATE, "invalid plan handle");
    if (!tile_select) return fail(XCORR_ERR_ARG, "null tile selection");
    xcorr_status s = check_ptr(d_out, "d_out");
    if (s != XCORR_OK) return s;
    const int nr = (p->d.n_inputs + kRowBlock - 1) / kRowBlock;
    const size_t nsel = (size_t)nr * (nr + 1) / 2;
    hipError_t e = hipSuccess;
    if (!p->d_tile_sel) e = hipMalloc((void**)&p->d_tile_sel, nsel);
    if (e != hipSuccess) {
        p->d_tile_sel = nullptr;
        (void)hipGetLastError();
        return fail(XCORR_ERR_NOMEM, "tile selection: %s", hipGetErrorString(e));
    }
    e = hipMemcpyAsync(p->d_tile_sel, tile_select, nsel, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = launch_dump_tiles(d_out, p->acc, p->acc_valid ? 1 : 0, p->acc32_valid ? p->acc32 : nullptr,
                              p->d_tile_sel, p->d.n_inputs, p->d.n_channels,
                              (int)(2 * elem_bytes(&p->d)), reset ? 1 : 0, p->stream);
    if (e != hipSuccess) return hip_fail(e, "tile dump");
    p->n_dumps += 1;
    fill_info(p, info);
    return XCORR_OK;
}

xcorr_status xcorr_corner_turn(const void* d_packets, const uint8_t* d_valid, const xcorr_packet_layout* L,
                               int32_t out_format, void* d_out, void* stream)
{
    if (!L) return fail(XCORR_ERR_ARG, "null layout");
    if (L->n_blocks < 1 || L->n_fengines < 1 || L->inputs_per_feng < 1 || L->n_channels < 1 ||
        L->spectra_per_packet < 1)
        return fail(XCORR_ERR_ARG, "every layout size must be >= 1");
    if (L->inputs_per_feng % 4) return fail(XCORR_ERR_UNSUPPORTED, "inputs_per_feng must be a multiple of 4");
    const int64_t n_in = (int64_t)L->n_fengines * L->inputs_per_feng;
    if (n_in > 32768) return fail(XCORR_ERR_UNSUPPORTED, "n_fengines * inputs_per_feng above 32768");
    if (out_format != XCORR_CI4 && out_format != XCORR_CI8) return fail(XCORR_ERR_ARG, "unknown out_format %d", out_format);
    xcorr_status s = check_ptr(d_packets, "d_packets");
    if (s == XCORR_OK) s = check_ptr(d_out, "d_out");
    if (s != XCORR_OK) return s;
    CornerTurnArgs a{};
    a.in = (const uint8_t*)d_packets;
    a.valid = d_valid;
    a.out = d_out;
    a.n_blocks = L->n_blocks;
    a.n_fengines = L->n_fengines;
    a.inputs_per_feng = L->inputs_per_feng;
    a.n_channels = L->n_channels;
    a.spectra = L->spectra_per_packet;
    a.n_inputs = (int32_t)n_in;
    a.n_time = (int64_t)L->n_blocks * L->spectra_per_packet;
    hipError_t e = launch_corner_turn(a, out_format, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "corner turn launch");
    return XCORR_OK;
}

namespace {

xcorr_status check_fstage_desc(const xcorr_fstage_desc* d, int64_t adc_stride, int64_t n_samples, int64_t* n_spec)
{
    if (!d) return fail(XCORR_ERR_ARG, "null descriptor");
    if (d->n_inputs < 1 || d->n_chan < 1) return fail(XCORR_ERR_ARG, "n_inputs and n_chan must be >= 1");
    if (d->n_points != 8192) return fail(XCORR_ERR_UNSUPPORTED, "n_points must be 8192");
    if (d->n_taps != 1 && d->n_taps != 2) return fail(XCORR_ERR_UNSUPPORTED, "n_taps must be 1 or 2");
    if (d->chan_begin < 0 || (int64_t)d->chan_begin + d->n_chan > d->n_points / 2)
        return fail(XCORR_ERR_ARG, "channels [%d, %d) outside [0, %d)", d->chan_begin, d->chan_begin + d->n_chan,
                    d->n_points / 2);
    if (d->out_kind != XCORR_FSTAGE_CI4 && d->out_kind != XCORR_FSTAGE_F32)
        return fail(XCORR_ERR_ARG, "unknown out_kind %d", d->out_kind);
    if (n_samples < 0 || adc_stride < n_samples || adc_stride % 2)
        return fail(XCORR_ERR_ARG, "need 0 <= n_samples <= adc_stride and an even adc_stride");
    *n_spec = std::max<int64_t>(0, n_samples / d->n_points - d->n_taps + 1);
    if (*n_spec > 0x7fffffff) return fail(XCORR_ERR_UNSUPPORTED, "too many spectra");
    return XCORR_OK;
}

}  // namespace

xcorr_status xcorr_clock_probe(void* d_out, int64_t ticks, int32_t* wall_khz, void* stream)
{
    if (!d_out || ((uintptr_t)d_out & 7)) return fail(XCORR_ERR_ARG, "d_out must be a non-null 8-byte aligned pointer");
    if (ticks < 1 || ticks >= ((int64_t)1 << 32)) return fail(XCORR_ERR_ARG, "ticks out of range");
    if (wall_khz) {
        int dev = 0, khz = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess) return hip_fail(e, "wall clock rate");
        *wall_khz = khz;
    }
    hipError_t e = launch_clock_probe((unsigned long long*)d_out, (long long)ticks, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "clock probe launch");
    return XCORR_OK;
}

xcorr_status xcorr_fstage_work_bytes(const xcorr_fstage_desc* d, int64_t n_samples, size_t* bytes)
{
    int64_t n_spec = 0;
    xcorr_status s = check_fstage_desc(d, n_samples + (n_samples & 1), n_samples, &n_spec);
    if (s != XCORR_OK) return s;
    if (!bytes) return fail(XCORR_ERR_ARG, "null bytes");
    *bytes = d->out_kind == XCORR_FSTAGE_CI4 ? (size_t)fstage_work_bytes(d->n_inputs, n_spec, d->chan_begin, d->n_chan)
                                             : 0;
    return XCORR_OK;
}

xcorr_status xcorr_fstage(const xcorr_fstage_desc* d, const void* d_adc, int64_t adc_stride, int64_t n_samples,
                          const float* d_coeff, const float* d_gain, void* d_work, void* d_out, int64_t* n_spectra,
                          void* stream)
{
    int64_t n_spec = 0;
    xcorr_status s0 = check_fstage_desc(d, adc_stride, n_samples, &n_spec);
    if (s0 != XCORR_OK) return s0;
    if (n_spectra) *n_spectra = n_spec;
    if (n_spec == 0) return XCORR_OK;
    xcorr_status s = check_ptr(d_adc, "d_adc");
    if (s == XCORR_OK) s = check_ptr(d_coeff, "d_coeff");
    if (s == XCORR_OK) s = check_ptr(d_gain, "d_gain");
    if (s == XCORR_OK) s = check_ptr(d_out, "d_out");
    if (s == XCORR_OK && d->out_kind == XCORR_FSTAGE_CI4) s = check_ptr(d_work, "d_work");
    if (s != XCORR_OK) return s;
    FstageArgs a{};
    a.adc = (const int8_t*)d_adc;
    a.adc_stride = adc_stride;
    a.coeff = d_coeff;
    a.gain = d_gain;
    a.out = d_out;
    a.work = d_work;
    a.n_inputs = d->n_inputs;
    a.n_taps = d->n_taps;
    a.n_spectra = (int32_t)n_spec;
    a.chan_begin = d->chan_begin;
    a.n_chan = d->n_chan;
    a.out_kind = d->out_kind;
    hipError_t e = launch_fstage(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "F-stage launch");
    return XCORR_OK;
}

xcorr_status xcorr_destroy(xcorr_plan_t p)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (p == nullptr || g_live.erase(p) == 0) return fail(XCORR_ERR_STATE, "invalid plan handle");
    }
    hipError_t e = hipStreamSynchronize(p->stream);
    release(p->acc);
    release(p->acc32);
    release(p->d_items);
    release(p->d_counters);
    release(p->d_tile_sel);
    release(p->d_pad);
    release(p->d_gate_buf);
    release(p->d_gate_idx);
    delete p;
    if (e != hipSuccess) return hip_fail(e, "destroy: stream synchronize");
    return XCORR_OK;
}

}  // extern "C"
