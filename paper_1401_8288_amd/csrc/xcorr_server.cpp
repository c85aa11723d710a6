// Streaming server: admission of integration streams by device memory and
// continuous batching of their windows into persistent int8 launches.  See
// include/xcorr.h.
#include "xcorr_host.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace xcorr;

namespace {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Window {
    int64_t ticket;
    const void* d_in;
    int64_t n_time;
    void* d_out;
};

struct Ticket {
    bool done = false;
    xcorr_status status = XCORR_OK;
    double t_submit = 0, t_done = 0;
    double cmac = 0;
    xcorr_dump_info info{};
};

struct Stream {
    xcorr_plan_desc desc{};
    size_t bytes = 0;
    xcorr_plan_t plan = nullptr;    // null until admitted
    bool closing = false;
    bool released = false;
    std::deque<Window> pending;
    int inflight = 0;               // windows of this stream on the GPU
};

struct Launch {
    hipEvent_t done = nullptr;
    std::vector<int64_t> tickets;
    std::vector<int32_t> sids;
    std::vector<xcorr_dump_info> info;
    xcorr_status status = XCORR_OK;
};

}  // namespace

struct xcorr_server_s {
    xcorr_server_desc d{};
    int device = 0;
    int n_cu = 256;
    hipStream_t stream = nullptr;
    int* d_counters = nullptr;

    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    std::map<int32_t, Stream> streams;
    std::deque<int32_t> waiting;
    int32_t next_sid = 1;
    std::unordered_map<int64_t, Ticket> tickets;
    int64_t next_ticket = 1;
    std::deque<Launch> inflight;
    size_t bytes_held = 0;
    int admitted = 0;
    bool stop = false;
    std::thread worker;

    int64_t windows_done = 0, launches = 0, batched_windows = 0;
    double cmac = 0, first_submit = -1, last_done = 0;
    std::vector<double> latencies;
};

namespace {

std::mutex g_mu;
std::set<xcorr_server_t> g_servers;

bool server_live(xcorr_server_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return s && g_servers.count(s);
}

// Admit waiting streams in arrival order while slots and budget allow.
// Called by the worker with the lock held.
void admit_locked(xcorr_server_t s)
{
    while (!s->waiting.empty()) {
        const int32_t sid = s->waiting.front();
        Stream& st = s->streams[sid];
        if (s->admitted >= s->d.max_streams || s->bytes_held + st.bytes > s->d.device_budget) break;
        xcorr_plan_desc pd = st.desc;
        pd.stream = s->stream;
        xcorr_plan_t p = nullptr;
        const xcorr_status rc = xcorr_plan(&p, &pd);
        if (rc != XCORR_OK) break;     // device memory short of the budget: retry later
        st.plan = p;
        s->bytes_held += st.bytes;
        s->admitted += 1;
        s->waiting.pop_front();
    }
}

// Release closed streams that have nothing queued or running (lock held).
void release_closed_locked(xcorr_server_t s)
{
    for (auto& kv : s->streams) {
        Stream& st = kv.second;
        if (st.closing && !st.released && st.plan && st.pending.empty() && st.inflight == 0) {
            (void)xcorr_destroy(st.plan);
            st.plan = nullptr;
            st.released = true;
            s->bytes_held -= st.bytes;
            s->admitted -= 1;
        }
    }
}

bool pending_admitted_locked(xcorr_server_t s)
{
    for (auto& kv : s->streams)
        if (kv.second.plan && !kv.second.pending.empty()) return true;
    return false;
}

bool pending_any_locked(xcorr_server_t s)
{
    for (auto& kv : s->streams)
        if (!kv.second.pending.empty()) return true;
    return false;
}

// Enqueues one batched launch of the given windows (lock not held).
xcorr_status launch_windows(xcorr_server_t s, const std::vector<xcorr_plan_t>& plans,
                            const std::vector<Window>& ws, Launch& L)
{
    // one persistent launch per (format, staging) group
    std::map<int, std::vector<size_t>> groups;
    for (size_t k = 0; k < plans.size(); ++k) {
        const xcorr_plan_s* p = plans[k];
        const int key = p->d.format == XCORR_CI8 ? 2 : (p->n_cols % 16 == 0 ? 0 : 1);
        groups[key].push_back(k);
    }
    L.info.assign(plans.size(), xcorr_dump_info{});
    for (auto& g : groups) {
        std::vector<xcorr_plan_t> gp;
        std::vector<const void*> in;
        std::vector<int64_t> nt;
        std::vector<void*> out;
        for (size_t k : g.second) {
            gp.push_back(plans[k]);
            in.push_back(ws[k].d_in);
            nt.push_back(ws[k].n_time);
            out.push_back(ws[k].d_out);
        }
        xcorr_batch_config cfg{g.first == 0 ? kTileDma4 : kTileRegs, ((s->n_cu + 7) / 8) * 8, 1, 0};
        std::vector<xcorr_dump_info> info;
        xcorr_status rc = run_fused_windows(s->stream, s->d_counters, cfg, gp, in, nt, out, info);
        if (rc != XCORR_OK) return rc;
        for (size_t j = 0; j < g.second.size(); ++j) L.info[g.second[j]] = info[j];
    }
    hipError_t e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(L.done, s->stream);
    if (e != hipSuccess) return hip_fail(e, "server event");
    return XCORR_OK;
}

void worker_main(xcorr_server_t s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        admit_locked(s);
        if (pending_admitted_locked(s) && (int)s->inflight.size() < s->d.max_inflight) {
            // continuous batching: the oldest window of every admitted stream
            std::vector<xcorr_plan_t> plans;
            std::vector<Window> ws;
            Launch L;
            for (auto& kv : s->streams) {
                Stream& st = kv.second;
                if (!st.plan || st.pending.empty()) continue;
                plans.push_back(st.plan);
                ws.push_back(st.pending.front());
                st.pending.pop_front();
                st.inflight += 1;
                L.tickets.push_back(ws.back().ticket);
                L.sids.push_back(kv.first);
            }
            s->launches += 1;
            s->batched_windows += (int64_t)ws.size();
            lk.unlock();
            L.status = launch_windows(s, plans, ws, L);
            if (L.status != XCORR_OK && !L.done) {
                // nothing to wait for: complete the tickets with the error now
                (void)hipStreamSynchronize(s->stream);
            }
            lk.lock();
            s->inflight.push_back(std::move(L));
            continue;
        }
        if (!s->inflight.empty()) {
            Launch L = std::move(s->inflight.front());
            s->inflight.pop_front();
            lk.unlock();
            if (L.done) {
                hipError_t e = hipEventSynchronize(L.done);
                if (e != hipSuccess && L.status == XCORR_OK) L.status = XCORR_ERR_DEVICE;
                (void)hipEventDestroy(L.done);
            }
            const double t = now_ms();
            lk.lock();
            for (size_t k = 0; k < L.tickets.size(); ++k) {
                Ticket& tk = s->tickets[L.tickets[k]];
                tk.done = true;
                tk.status = L.status;
                tk.t_done = t;
                tk.info = L.info.empty() ? xcorr_dump_info{} : L.info[k];
                s->streams[L.sids[k]].inflight -= 1;
                if (L.status == XCORR_OK) {
                    s->windows_done += 1;
                    s->cmac += tk.cmac;
                    s->latencies.push_back(t - tk.t_submit);
                    s->last_done = t;
                }
            }
            release_closed_locked(s);
            s->cv_done.notify_all();
            continue;
        }
        release_closed_locked(s);
        if (s->stop && !pending_any_locked(s)) break;
        if (s->stop && s->admitted == 0 && !s->waiting.empty() && !pending_admitted_locked(s)) {
            // streams that can never be admitted (device memory below the
            // budget): fail their windows so that destroy returns
            for (auto& kv : s->streams)
                for (const Window& w : kv.second.pending) {
                    Ticket& tk = s->tickets[w.ticket];
                    tk.done = true;
                    tk.status = XCORR_ERR_NOMEM;
                }
            for (auto& kv : s->streams) kv.second.pending.clear();
            s->cv_done.notify_all();
            break;
        }
        s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
    }
}

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

xcorr_status xcorr_server_create(xcorr_server_t* out, const xcorr_server_desc* d)
{
    if (!out || !d) return fail(XCORR_ERR_ARG, "null argument");
    if (d->max_streams < 1 || d->max_streams > 64) return fail(XCORR_ERR_ARG, "max_streams must be 1..64");
    if (d->max_inflight < 1 || d->max_inflight > 8) return fail(XCORR_ERR_ARG, "max_inflight must be 1..8");
    if (d->device_budget == 0) return fail(XCORR_ERR_ARG, "zero device budget");
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    xcorr_server_t s = new (std::nothrow) xcorr_server_s();
    if (!s) return fail(XCORR_ERR_NOMEM, "host allocation");
    s->d = *d;
    s->device = dev;
    s->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    s->stream = (hipStream_t)d->stream;
    e = hipMalloc((void**)&s->d_counters, kCounterInts * sizeof(int));
    if (e == hipSuccess) e = hipMemset(s->d_counters, 0, kCounterInts * sizeof(int));
    if (e != hipSuccess) {
        if (s->d_counters) (void)hipFree(s->d_counters);
        delete s;
        (void)hipGetLastError();
        return fail(XCORR_ERR_NOMEM, "server counters: %s", hipGetErrorString(e));
    }
    s->worker = std::thread(worker_main, s);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_servers.insert(s);
    }
    *out = s;
    return XCORR_OK;
}

xcorr_status xcorr_server_open(xcorr_server_t s, const xcorr_plan_desc* desc, int32_t* sid)
{
    if (!server_live(s)) return fail(XCORR_ERR_STATE, "invalid server handle");
    if (!desc || !sid) return fail(XCORR_ERR_ARG, "null argument");
    if (desc->path != XCORR_PATH_I8_MFMA) return fail(XCORR_ERR_UNSUPPORTED, "the server runs the int8 path");
    size_t bytes = 0;
    xcorr_status rc = xcorr_plan_bytes(desc, &bytes);
    if (rc != XCORR_OK) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(XCORR_ERR_STATE, "server is shutting down");
    if (bytes > s->d.device_budget)
        return fail(XCORR_ERR_NOMEM, "stream needs %zu bytes, budget is %zu", bytes, s->d.device_budget);
    const int32_t id = s->next_sid++;
    Stream& st = s->streams[id];
    st.desc = *desc;
    st.bytes = bytes;
    s->waiting.push_back(id);
    *sid = id;
    s->cv_work.notify_all();
    return XCORR_OK;
}

xcorr_status xcorr_server_submit(xcorr_server_t s, int32_t sid, const void* d_in, int64_t n_time, void* d_out,
                                 int64_t* ticket)
{
    if (!server_live(s)) return fail(XCORR_ERR_STATE, "invalid server handle");
    if (!ticket) return fail(XCORR_ERR_ARG, "null ticket");
    if (n_time <= 0) return fail(XCORR_ERR_ARG, "a window needs n_time > 0");
    xcorr_status rc = check_ptr(d_in, "d_in");
    if (rc == XCORR_OK) rc = check_ptr(d_out, "d_out");
    if (rc != XCORR_OK) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->streams.find(sid);
    if (it == s->streams.end() || it->second.closing) return fail(XCORR_ERR_ARG, "unknown or closed stream %d", sid);
    if ((it->second.desc.flags & XCORR_FLAG_OUT_I32) && n_time > fold_bound_of(&it->second.desc))
        return fail(XCORR_ERR_ARG, "int32 output: window of %lld samples past the bound", (long long)n_time);
    const int64_t t = s->next_ticket++;
    Ticket& tk = s->tickets[t];
    tk.t_submit = now_ms();
    const xcorr_plan_desc& pd = it->second.desc;
    tk.cmac = (double)pd.n_inputs * (pd.n_inputs + 1) / 2 * pd.n_channels * (double)n_time;
    if (s->first_submit < 0) s->first_submit = tk.t_submit;
    it->second.pending.push_back(Window{t, d_in, n_time, d_out});
    *ticket = t;
    s->cv_work.notify_all();
    return XCORR_OK;
}

xcorr_status xcorr_server_poll(xcorr_server_t s, int64_t ticket, int32_t* done, xcorr_dump_info* info,
                               double* latency_ms)
{
    if (!server_live(s)) return fail(XCORR_ERR_STATE, "invalid server handle");
    if (!done) return fail(XCORR_ERR_ARG, "null done");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(XCORR_ERR_ARG, "unknown ticket %lld", (long long)ticket);
    *done = it->second.done ? 1 : 0;
    if (it->second.done) {
        if (info) *info = it->second.info;
        if (latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
        if (it->second.status != XCORR_OK) return fail(it->second.status, "window failed");
    }
    return XCORR_OK;
}

xcorr_status xcorr_server_wait(xcorr_server_t s, int64_t ticket, xcorr_dump_info* info, double* latency_ms)
{
    if (!server_live(s)) return fail(XCORR_ERR_STATE, "invalid server handle");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(XCORR_ERR_ARG, "unknown ticket %lld", (long long)ticket);
    s->cv_done.wait(lk, [&] { return s->tickets[ticket].done; });
    const Ticket& tk = s->tickets[ticket];
    if (info) *info = tk.info;
    if (latency_ms) *latency_ms = tk.t_done - tk.t_submit;
    if (tk.status != XCORR_OK) return fail(tk.status, "window failed");
    return XCORR_OK;
}

xcorr_status xcorr_server_close(xcorr_server_t s, int32_t sid)
{
    if (!server_live(s)) return fail(XCORR_ERR_STATE, "invalid server handle");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->streams.find(sid);
    if (it == s->streams.end() || it->second.closing) return fail(XCORR_ERR_ARG, "unknown or closed stream %d", sid);
    it->second.closing = true;
    s->cv_work.notify_all();
    return XCORR_OK;
}

xcorr_status xcorr_server_query(xcorr_server_t s, xcorr_server_stats* st)
{
    if (!server_live(s)) return fail(XCORR_ERR_STATE, "invalid server handle");
    if (!st) return fail(XCORR_ERR_ARG, "null stats");
    std::lock_guard<std::mutex> lk(s->mu);
    st->windows_done = s->windows_done;
    st->launches = s->launches;
    st->cmac = s->cmac;
    st->elapsed_s = s->first_submit >= 0 && s->last_done > s->first_submit ? (s->last_done - s->first_submit) / 1e3 : 0;
    st->latency_p50_ms = percentile(s->latencies, 0.50);
    st->latency_p99_ms = percentile(s->latencies, 0.99);
    st->latency_max_ms = s->latencies.empty() ? 0 : *std::max_element(s->latencies.begin(), s->latencies.end());
    st->mean_batch = s->launches ? (double)s->batched_windows / s->launches : 0;
    st->streams_admitted = s->admitted;
    st->streams_waiting = (int32_t)s->waiting.size();
    st->device_bytes = s->bytes_held;
    return XCORR_OK;
}

xcorr_status xcorr_server_destroy(xcorr_server_t s)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!s || g_servers.erase(s) == 0) return fail(XCORR_ERR_STATE, "invalid server handle");
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto& kv : s->streams) kv.second.closing = true;
        s->cv_work.notify_all();
    }
    s->worker.join();
    hipError_t e = hipStreamSynchronize(s->stream);
    for (auto& kv : s->streams)
        if (kv.second.plan) (void)xcorr_destroy(kv.second.plan);
    (void)hipFree(s->d_counters);
    delete s;
    if (e != hipSuccess) return hip_fail(e, "server destroy: stream synchronize");
    return XCORR_OK;
}

}  // extern "C"
