// Batches of plans: one persistent int8 launch per time chunk for several
// subarrays, the autotuner that picks the launch configuration, and hipGraph
// capture of a whole integration step.  See include/xcorr.h.
#include "xcorr_host.h"
#include "xcorr_gate.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <vector>

using namespace xcorr;

struct xcorr_batch_s {
    std::vector<xcorr_plan_t> plans;
    hipStream_t stream = nullptr;
    int format = 0;
    bool dma_ok = false;            // every plan allows the LDS-DMA tiles
    int n_cu = 256;
    int* d_counters = nullptr;      // kCounterInts work-queue counters
    xcorr_batch_config cfg{};
};

struct xcorr_graph_s {
    xcorr_batch_t batch = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int64_t> n_time;
};

namespace {

std::mutex g_mu;
std::set<xcorr_batch_t> g_batches;
std::set<xcorr_graph_t> g_graphs;

bool batch_live(xcorr_batch_t b)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return b && g_batches.count(b);
}

bool graph_live(xcorr_graph_t g)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g && g_graphs.count(g);
}

// One (plan, time chunk) of a step.
struct Entry {
    LaunchArgs a;
    int64_t t_len;
    const xcorr_plan_s* plan;
};

// Per-XCD slices of the global item list.  balance = 1: cut at channel-group
// boundaries so that the slices carry equal cost (MFMA blocks x samples);
// balance = 0: equal item counts.
void make_slices(const std::vector<Entry>& es, const int* first, int n_blocks, int balance, int32_t* slice)
{
    slice[0] = 0;
    slice[8] = n_blocks;
    if (!balance) {
        const int per = (n_blocks + 7) / 8;
        for (int x = 1; x < 8; ++x) slice[x] = std::min(n_blocks, x * per);
        return;
    }
    // cost of each channel group of each entry, in order
    std::vector<std::pair<int, double>> groups;   // (first item of the group, cost)
    double total = 0;
    for (size_t e = 0; e < es.size(); ++e) {
        const xcorr_plan_s* p = es[e].plan;
        const std::vector<WorkItem>& its = p->h_items;
        const int n_items = es[e].a.n_items;
        double gc = 0;
        for (const WorkItem& it : its) gc += item_blocks(it);
        gc *= (double)es[e].t_len;
        for (int g = 0; g < es[e].a.n_blocks / n_items; ++g) {
            groups.emplace_back(first[e] + g * n_items, gc);
            total += gc;
        }
    }
    double acc = 0;
    size_t gi = 0;
    for (int x = 1; x < 8; ++x) {
        const double target = total * x / 8;
        while (gi < groups.size() && acc + groups[gi].second * 0.5 < target) acc += groups[gi++].second;
        slice[x] = gi < groups.size() ? groups[gi].first : n_blocks;
        slice[x] = std::max(slice[x], slice[x - 1]);
    }
}

xcorr_status launch_entries_same_width(xcorr_batch_t b, const std::vector<Entry>& es, const xcorr_batch_config& cfg);

// Entries of different result modes (LaunchArgs.out32) go out as one
// launch per mode.
xcorr_status launch_entries(xcorr_batch_t b, const std::vector<Entry>& es, const xcorr_batch_config& cfg)
{
    std::vector<Entry> by_mode[3];
    for (const Entry& e : es) by_mode[e.a.out32].push_back(e);
    for (int m = 0; m < 3; ++m) {
        if (by_mode[m].empty()) continue;
        xcorr_status s = launch_entries_same_width(b, by_mode[m], cfg);
        if (s != XCORR_OK) return s;
    }
    return XCORR_OK;
}

xcorr_status launch_entries_same_width(xcorr_batch_t b, const std::vector<Entry>& es, const xcorr_batch_config& cfg)
{
    for (size_t e0 = 0; e0 < es.size(); e0 += kMaxBatchEntries) {
        const size_t n = std::min<size_t>(kMaxBatchEntries, es.size() - e0);
        BatchArgs ba;
        std::memset(&ba, 0, sizeof ba);
        std::vector<Entry> part(es.begin() + e0, es.begin() + e0 + n);
        ba.n_entries = (int)n;
        ba.xcd_map = 1;
        int total = 0;
        for (size_t e = 0; e < n; ++e) {
            ba.first[e] = total;
            ba.e[e] = part[e].a;
            total += part[e].a.n_blocks;
        }
        ba.first[n] = total;
        ba.n_blocks = total;
        ba.counters = b->d_counters;
        make_slices(part, ba.first, total, cfg.balance, ba.slice);
        hipError_t err = launch_i8_batch(ba, b->format, cfg.tile, cfg.grid, b->stream);
        if (err != hipSuccess) return hip_fail(err, "batch launch");
    }
    return XCORR_OK;
}

// Enqueues one step.  fused_to_acc: time every plan as a fused window whose
// result lands in its own accumulator (autotuner); plan state is not changed.
xcorr_status run_step(xcorr_batch_t b, const void* const* d_in, const int64_t* n_time, void* const* d_out,
                      const int32_t* reset, xcorr_dump_info* info, const xcorr_batch_config& cfg,
                      bool fused_to_acc)
{
    const size_t np = b->plans.size();
    // a plan may appear more than once (the server's windows of one
    // stream) only where it reads the caller's rows as they are: staged
    // rows would share the plan's one pad buffer
    for (size_t k = 0; k < np; ++k)
        for (size_t j = 0; j < k; ++j)
            if (b->plans[j] == b->plans[k] && b->plans[k]->n_cols != b->plans[k]->d.n_inputs)
                return fail(XCORR_ERR_UNSUPPORTED, "a plan with padded rows twice in one step");
    std::vector<int64_t> chunks(np, 0);
    int64_t rounds = 0;
    for (size_t k = 0; k < np; ++k) {
        const xcorr_plan_s* p = b->plans[k];
        chunks[k] = n_time[k] > 0 ? (n_time[k] + p->fold_bound - 1) / p->fold_bound : 0;
        rounds = std::max(rounds, chunks[k]);
    }
    // fused_to_acc: every chunk writes (the first) or adds to the plan's own
    // accumulator in its result type, from an empty state
    std::vector<AccState> st(np);
    for (size_t k = 0; k < np; ++k) st[k] = fused_to_acc ? AccState{false, false, 0} : acc_state(b->plans[k]);
    for (int64_t r = 0; r < rounds; ++r) {
        std::vector<Entry> es;
        for (size_t k = 0; k < np; ++k) {
            if (r >= chunks[k]) continue;
            xcorr_plan_s* p = b->plans[k];
            const int64_t row = row_bytes_of(p);
            const int64_t t0 = r * p->fold_bound;
            const int64_t len = std::min<int64_t>(p->fold_bound, n_time[k] - t0);
            const bool last = r == chunks[k] - 1;
            ChunkTarget t;
            if (fused_to_acc) {
                t = ChunkTarget{st[k].acc_valid ? p->acc : nullptr, p->acc, p->out32, false, false};
                st[k].acc_valid = true;
            } else {
                void* fin = (last && d_out[k] && reset && reset[k]) ? d_out[k] : nullptr;
                t = chunk_target(p, st[k], len, fin);
            }
            if (t.fold) {
                // the plan's int32 accumulator is full: fold it first (its
                // own launch; windows past the fold bound only)
                hipError_t e = fold_acc32(p, t.fold_acc_valid, b->stream);
                if (e != hipSuccess) return hip_fail(e, "int32 accumulator fold");
            }
            const uint8_t* cin = (const uint8_t*)d_in[k] + t0 * row;
            int64_t cstride = row * n_time[k];
            xcorr_status ss = stage_chunk(p, cin, cstride, len, b->stream, &cin, &cstride);
            if (ss != XCORR_OK) return ss;
            Entry en;
            en.a = chunk_args(p, cin, cstride, (int32_t)len, t.src, t.dst, t.mode);
            en.t_len = len;
            en.plan = p;
            es.push_back(en);
        }
        xcorr_status s = launch_entries(b, es, cfg);
        if (s != XCORR_OK) return s;
    }
    if (fused_to_acc) return XCORR_OK;
    // dumps that were not fused into the last launch, and bookkeeping
    for (size_t k = 0; k < np; ++k) {
        xcorr_plan_s* p = b->plans[k];
        const bool dump = d_out[k] != nullptr;
        const bool rst = dump && reset && reset[k];
        const bool fused = dump && rst && n_time[k] > 0;
        set_acc_state(p, st[k]);
        if (dump && !fused) {
            hipError_t e = launch_dump_of(p, d_out[k], b->stream);
            if (e != hipSuccess) return hip_fail(e, "batch dump");
        }
        p->samples += n_time[k];
        p->total += n_time[k];
        if (dump) {
            p->n_dumps += 1;
            if (info) fill_info(p, &info[k]);
        }
        if (rst) {
            reset_acc(p);
            p->samples = 0;
            p->window_start = p->total;
        }
    }
    return XCORR_OK;
}

xcorr_status check_step(xcorr_batch_t b, const void* const* d_in, const int64_t* n_time, void* const* d_out)
{
    if (!d_in || !n_time) return fail(XCORR_ERR_ARG, "null input arrays");
    for (size_t k = 0; k < b->plans.size(); ++k) {
        if (!plan_live(b->plans[k])) return fail(XCORR_ERR_STATE, "plan %zu of the batch was destroyed", k);
        if (n_time[k] < 0) return fail(XCORR_ERR_ARG, "negative n_time for plan %zu", k);
        if (n_time[k] > 0) {
            xcorr_status s = check_ptr(d_in[k], "d_in[k]");
            if (s == XCORR_OK) s = check_window(b->plans[k], n_time[k]);
            if (s != XCORR_OK) return s;
        }
        if (d_out && d_out[k]) {
            xcorr_status s = check_ptr(d_out[k], "d_out[k]");
            if (s != XCORR_OK) return s;
        }
    }
    return XCORR_OK;
}

xcorr_status check_config(xcorr_batch_t b, const xcorr_batch_config& c)
{
    if (c.tile < 0 || c.tile > kTileRegs) return fail(XCORR_ERR_ARG, "unknown tile %d", c.tile);
    if ((c.tile == kTileDma8 || c.tile == kTileDma4) && !b->dma_ok)
        return fail(XCORR_ERR_UNSUPPORTED, "LDS-DMA tiles need rows of a multiple of 16 inputs");
    if (c.tile == kTileDma8 && b->format != XCORR_CI4)
        return fail(XCORR_ERR_UNSUPPORTED, "the DMA8 tile takes 4-bit samples only");
    if (c.grid < 8 || c.grid % 8 || c.grid > 65536) return fail(XCORR_ERR_ARG, "grid must be a multiple of 8");
    if (c.balance != 0 && c.balance != 1) return fail(XCORR_ERR_ARG, "balance must be 0 or 1");
    return XCORR_OK;
}

}  // namespace

namespace xcorr {

xcorr_status run_fused_windows(hipStream_t stream, int* d_counters, const xcorr_batch_config& cfg,
                               const std::vector<xcorr_plan_t>& plans, const std::vector<const void*>& d_in,
                               const std::vector<int64_t>& n_time, const std::vector<void*>& d_out,
                               std::vector<xcorr_dump_info>& info)
{
    xcorr_batch_s tmp;
    tmp.plans = plans;
    tmp.stream = stream;
    tmp.format = plans.empty() ? 0 : plans[0]->d.format;
    tmp.d_counters = d_counters;
    std::vector<int32_t> resets(plans.size(), 1);
    info.resize(plans.size());
    return run_step(&tmp, d_in.data(), n_time.data(), d_out.data(), resets.data(), info.data(), cfg, false);
}

}  // namespace xcorr

extern "C" {

xcorr_status xcorr_batch_create(xcorr_batch_t* out, const xcorr_plan_t* plans, int32_t n_plans, void* stream)
{
    if (!out || !plans) return fail(XCORR_ERR_ARG, "null argument");
    if (n_plans < 1 || n_plans > 64) return fail(XCORR_ERR_ARG, "n_plans must be 1..64");
    int fmt = -1;
    bool dma_ok = true;
    for (int k = 0; k < n_plans; ++k) {
        if (!plan_live(plans[k])) return fail(XCORR_ERR_STATE, "plan %d is not valid", k);
        const xcorr_plan_s* p = plans[k];
        if (p->d.path != XCORR_PATH_I8_MFMA) return fail(XCORR_ERR_UNSUPPORTED, "batches use the int8 path");
        if (fmt >= 0 && p->d.format != fmt) return fail(XCORR_ERR_ARG, "plans of a batch must share the format");
        fmt = p->d.format;
        dma_ok = dma_ok && p->n_cols % 16 == 0;
        for (int j = 0; j < k; ++j)
            if (plans[j] == plans[k]) return fail(XCORR_ERR_ARG, "plan %d appears twice", k);
    }
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    xcorr_batch_t b = new (std::nothrow) xcorr_batch_s();
    if (!b) return fail(XCORR_ERR_NOMEM, "host allocation");
    b->plans.assign(plans, plans + n_plans);
    b->stream = (hipStream_t)stream;
    b->format = fmt;
    b->dma_ok = dma_ok;
    b->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    b->cfg.tile = dma_ok ? kTileDma4 : kTileRegs;
    b->cfg.grid = ((b->n_cu + 7) / 8) * 8;
    b->cfg.balance = 1;
    e = hipMalloc((void**)&b->d_counters, kCounterInts * sizeof(int));
    if (e == hipSuccess) e = hipMemset(b->d_counters, 0, kCounterInts * sizeof(int));
    if (e != hipSuccess) {
        if (b->d_counters) (void)hipFree(b->d_counters);
        delete b;
        (void)hipGetLastError();
        return fail(XCORR_ERR_NOMEM, "batch counters: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_batches.insert(b);
    }
    *out = b;
    return XCORR_OK;
}

xcorr_status xcorr_batch_run(xcorr_batch_t b, const void* const* d_in, const int64_t* n_time, void* const* d_out,
                             const int32_t* reset, xcorr_dump_info* info)
{
    if (!batch_live(b)) return fail(XCORR_ERR_STATE, "invalid batch handle");
    xcorr_status s = check_step(b, d_in, n_time, d_out);
    if (s != XCORR_OK) return s;
    std::vector<void*> outs(b->plans.size(), nullptr);
    if (d_out) outs.assign(d_out, d_out + b->plans.size());
    return run_step(b, d_in, n_time, outs.data(), reset, info, b->cfg, false);
}

xcorr_status xcorr_batch_get_config(xcorr_batch_t b, xcorr_batch_config* c)
{
    if (!batch_live(b)) return fail(XCORR_ERR_STATE, "invalid batch handle");
    if (!c) return fail(XCORR_ERR_ARG, "null config");
    *c = b->cfg;
    return XCORR_OK;
}

xcorr_status xcorr_batch_set_config(xcorr_batch_t b, const xcorr_batch_config* c)
{
    if (!batch_live(b)) return fail(XCORR_ERR_STATE, "invalid batch handle");
    if (!c) return fail(XCORR_ERR_ARG, "null config");
    xcorr_batch_config v = *c;
    if (v.tile == kTileDefault) v.tile = b->dma_ok ? kTileDma4 : kTileRegs;
    xcorr_status s = check_config(b, v);
    if (s != XCORR_OK) return s;
    b->cfg = v;
    return XCORR_OK;
}

xcorr_status xcorr_batch_autotune(xcorr_batch_t b, const void* const* d_in, const int64_t* n_time, int32_t reps,
                                  xcorr_batch_config* chosen, float* ms_best)
{
    if (!batch_live(b)) return fail(XCORR_ERR_STATE, "invalid batch handle");
    if (reps < 1 || reps > 1000) return fail(XCORR_ERR_ARG, "reps must be 1..1000");
    xcorr_status s = check_step(b, d_in, n_time, nullptr);
    if (s != XCORR_OK) return s;
    for (xcorr_plan_t p : b->plans)
        if (p->acc_valid || p->acc32_valid || p->samples != 0)
            return fail(XCORR_ERR_STATE, "autotune needs every plan freshly reset");
    std::vector<int> tiles;
    if (!b->dma_ok) tiles = {kTileRegs};
    else if (b->format == XCORR_CI4) tiles = {kTileDma4, kTileDma8, kTileRegs};
    else tiles = {kTileDma4, kTileRegs};
    const int g1 = ((b->n_cu + 7) / 8) * 8;
    std::vector<xcorr_batch_config> cands;
    for (int t : tiles)
        for (int g : {g1, 2 * g1})
            for (int bal : {1, 0}) cands.push_back(xcorr_batch_config{t, g, bal, 0});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "autotune events");
    float best = 0;
    xcorr_batch_config best_cfg = b->cfg;
    xcorr_status st = XCORR_OK;
    for (const xcorr_batch_config& c : cands) {
        st = run_step(b, d_in, n_time, nullptr, nullptr, nullptr, c, true);   // warm-up
        if (st != XCORR_OK) break;
        e = hipEventRecord(e0, b->stream);
        for (int r = 0; r < reps && e == hipSuccess && st == XCORR_OK; ++r)
            st = run_step(b, d_in, n_time, nullptr, nullptr, nullptr, c, true);
        if (st != XCORR_OK) break;
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = hip_fail(e, "autotune timing");
            break;
        }
        ms /= reps;
        if (best == 0 || ms < best) {
            best = ms;
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != XCORR_OK) return st;
    b->cfg = best_cfg;
    if (chosen) *chosen = best_cfg;
    if (ms_best) *ms_best = best;
    return XCORR_OK;
}

xcorr_status xcorr_batch_capture(xcorr_batch_t b, const void* const* d_in, const int64_t* n_time,
                                 void* const* d_out, xcorr_graph_t* out)
{
    if (!batch_live(b)) return fail(XCORR_ERR_STATE, "invalid batch handle");
    if (!out || !d_out) return fail(XCORR_ERR_ARG, "null argument");
    xcorr_status s = check_step(b, d_in, n_time, d_out);
    if (s != XCORR_OK) return s;
    const size_t np = b->plans.size();
    for (size_t k = 0; k < np; ++k) {
        if (n_time[k] <= 0 || !d_out[k]) return fail(XCORR_ERR_ARG, "a graph step needs n_time > 0 and d_out for every plan");
        if (b->plans[k]->acc_valid || b->plans[k]->acc32_valid)
            return fail(XCORR_ERR_STATE, "graph capture needs every plan freshly reset");
    }
    if (!b->stream) return fail(XCORR_ERR_ARG, "graph capture needs a non-null batch stream");
    xcorr_graph_t g = new (std::nothrow) xcorr_graph_s();
    if (!g) return fail(XCORR_ERR_NOMEM, "host allocation");
    g->batch = b;
    g->n_time.assign(n_time, n_time + np);
    // the step is recorded, not run: plan bookkeeping is restored afterwards
    std::vector<xcorr_plan_s> saved;
    for (xcorr_plan_t p : b->plans) saved.push_back(*p);
    std::vector<int32_t> resets(np, 1);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "begin capture");
    }
    s = run_step(b, d_in, n_time, d_out, resets.data(), nullptr, b->cfg, false);
    e = hipStreamEndCapture(b->stream, &g->graph);
    for (size_t k = 0; k < np; ++k) *b->plans[k] = saved[k];
    if (s == XCORR_OK && e != hipSuccess) s = hip_fail(e, "end capture");
    if (s == XCORR_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) s = hip_fail(e, "graph instantiate");
    }
    if (s != XCORR_OK) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return s;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_graphs.insert(g);
    }
    *out = g;
    return XCORR_OK;
}

xcorr_status xcorr_graph_launch(xcorr_graph_t g)
{
    if (!graph_live(g)) return fail(XCORR_ERR_STATE, "invalid graph handle");
    xcorr_batch_t b = g->batch;
    if (!batch_live(b)) return fail(XCORR_ERR_STATE, "the graph's batch was destroyed");
    // the replay writes every plan's bookkeeping (and, past the fold bound,
    // its accumulator): refuse it once any of them was destroyed
    for (size_t k = 0; k < b->plans.size(); ++k)
        if (!plan_live(b->plans[k])) return fail(XCORR_ERR_STATE, "plan %zu of the graph's batch was destroyed", k);
    hipError_t e = hipGraphLaunch(g->exec, b->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    for (size_t k = 0; k < b->plans.size(); ++k) {
        xcorr_plan_s* p = b->plans[k];
        p->total += g->n_time[k];
        p->n_dumps += 1;
        p->samples = 0;
        p->window_start = p->total;
        reset_acc(p);
    }
    return XCORR_OK;
}

xcorr_status xcorr_graph_destroy(xcorr_graph_t g)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g || g_graphs.erase(g) == 0) return fail(XCORR_ERR_STATE, "invalid graph handle");
    }
    hipError_t e = hipSuccess;
    if (batch_live(g->batch)) e = hipStreamSynchronize(g->batch->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    if (e != hipSuccess) return hip_fail(e, "graph destroy: stream synchronize");
    return XCORR_OK;
}

xcorr_status xcorr_accumulate_gated(const xcorr_plan_t* plans, int32_t n_gates, const void* d_in, int64_t n_time,
                                    const uint8_t* gate)
{
    if (!plans || n_gates < 1 || n_gates > 64) return fail(XCORR_ERR_ARG, "n_gates must be 1..64");
    if (n_time < 0) return fail(XCORR_ERR_ARG, "negative n_time");
    for (int g = 0; g < n_gates; ++g) {
        if (!plan_live(plans[g])) return fail(XCORR_ERR_STATE, "gate plan %d is not valid", g);
        const xcorr_plan_s* p = plans[g];
        const xcorr_plan_s* p0 = plans[0];
        if (p->d.n_inputs != p0->d.n_inputs || p->d.n_channels != p0->d.n_channels || p->d.format != p0->d.format ||
            p->stream != p0->stream)
            return fail(XCORR_ERR_ARG, "gate plans must share inputs, channels, format and stream");
        for (int h = 0; h < g; ++h)
            if (plans[h] == plans[g]) return fail(XCORR_ERR_ARG, "gate plan %d appears twice", g);
    }
    if (n_time == 0) return XCORR_OK;
    if (!gate) return fail(XCORR_ERR_ARG, "null gate array");
    xcorr_status st = check_ptr(d_in, "d_in");
    if (st != XCORR_OK) return st;
    for (int64_t t = 0; t < n_time; ++t)
        if (gate[t] != 0xFF && gate[t] >= n_gates) return fail(XCORR_ERR_ARG, "gate[%lld] out of range", (long long)t);
    {
        std::vector<int64_t> per(n_gates, 0);
        for (int64_t t = 0; t < n_time; ++t)
            if (gate[t] != 0xFF) per[gate[t]] += 1;
        for (int g = 0; g < n_gates; ++g) {
            st = check_window(plans[g], per[g]);
            if (st != XCORR_OK) return st;
        }
    }

    // The sample indices of each gate, in time order, in one list (gate g
    // at off[g] .. off[g] + cnt[g]) held by the first plan; each gate's plan
    // then accumulates those samples.
    xcorr_plan_s* p0 = plans[0];
    std::vector<int32_t> idx;
    std::vector<int64_t> off(n_gates, 0), cnt(n_gates, 0);
    for (int64_t t = 0; t < n_time; ++t)
        if (gate[t] != 0xFF) cnt[gate[t]] += 1;
    int64_t kept = 0;
    for (int g = 0; g < n_gates; ++g) {
        off[g] = kept;
        kept += cnt[g];
    }
    if (kept == 0) return XCORR_OK;
    if (kept > 0x7fffffff) return fail(XCORR_ERR_UNSUPPORTED, "window too long for gating");
    idx.resize(kept);
    {
        std::vector<int64_t> pos(off);
        for (int64_t t = 0; t < n_time; ++t)
            if (gate[t] != 0xFF) idx[pos[gate[t]]++] = (int32_t)t;
    }
    const int64_t row = row_bytes_of(p0), prow = staged_row_bytes(p0);
    // Persistent depth-4 LDS-DMA int8 plans read each gate's rows where they
    // are, through the gate's list of sample indices (its launches copy the
    // listed rows straight into LDS); other plans read a packed copy.
    bool listed = true;
    for (int g = 0; g < n_gates; ++g) listed = listed && row_list_cap(plans[g], row * n_time) > 0;
    xcorr_status gs = grow_buffer(p0, p0->stream, (void**)&p0->d_gate_idx, &p0->gate_idx_bytes, (size_t)kept * 4,
                                  "gated sample indices");
    if (gs == XCORR_OK && !listed)
        gs = grow_buffer(p0, p0->stream, &p0->d_gate_buf, &p0->gate_buf_bytes, (size_t)kept * prow * p0->d.n_channels,
                         "gated samples");
    if (gs != XCORR_OK) return gs;
    hipError_t e = hipMemcpyAsync(p0->d_gate_idx, idx.data(), (size_t)kept * 4, hipMemcpyHostToDevice, p0->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p0->stream);   // idx is a host temporary
    if (e != hipSuccess) return hip_fail(e, "gate indices");
    if (listed) {
        for (int g = 0; g < n_gates; ++g) {
            if (cnt[g] == 0) continue;
            st = run_window_rows(plans[g], (const uint8_t*)d_in, row * n_time, p0->d_gate_idx + off[g], cnt[g]);
            if (st != XCORR_OK) return st;
        }
        for (int g = 0; g < n_gates; ++g) {
            plans[g]->samples += cnt[g];
            plans[g]->total += cnt[g];
        }
        return XCORR_OK;
    }
    // rows of the packed buffer: the kernels' row width (zero padded when
    // the plans' rows need it), so the gates' launches read it as it is
    e = prow == row ? launch_gather_rows(p0->d_gate_buf, d_in, p0->d_gate_idx, kept, n_time, row, p0->d.n_channels,
                                         p0->stream)
                    : launch_pad_rows((uint8_t*)p0->d_gate_buf, (int)prow, (const uint8_t*)d_in, (int)row,
                                      row * n_time, p0->d_gate_idx, kept, p0->d.n_channels, p0->stream);
    if (e != hipSuccess) return hip_fail(e, "gate gather");

    // One launch (per fold chunk) per gate, each over all channels: a gate
    // with few samples is bound by its accumulator's read and write, and a
    // launch of its own spreads that traffic over the whole chip.
    const uint8_t* packed = (const uint8_t*)p0->d_gate_buf;
    for (int g = 0; g < n_gates; ++g) {
        if (cnt[g] == 0) continue;
        st = run_window_strided(plans[g], packed + off[g] * prow, prow * kept, cnt[g], nullptr, true);
        if (st != XCORR_OK) return st;
    }
    for (int g = 0; g < n_gates; ++g) {
        plans[g]->samples += cnt[g];
        plans[g]->total += cnt[g];
    }
    return XCORR_OK;
}

xcorr_status xcorr_batch_destroy(xcorr_batch_t b)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!b || g_batches.erase(b) == 0) return fail(XCORR_ERR_STATE, "invalid batch handle");
    }
    hipError_t e = hipStreamSynchronize(b->stream);
    (void)hipFree(b->d_counters);
    delete b;
    if (e != hipSuccess) return hip_fail(e, "batch destroy: stream synchronize");
    return XCORR_OK;
}

}  // extern "C"
