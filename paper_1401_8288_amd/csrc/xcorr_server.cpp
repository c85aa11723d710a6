// Streaming server: admission of integration streams by device memory and
// continuous batching of their windows into persistent int8 launches.  See
// include/xcorr.h.
#include "xcorr_host.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <cstdio>
#include <set>
#include <sstream>
#include <string>
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
    double deadline;                // ms on the steady clock; infinity = none
    double cmac;
};

struct Ticket {
    bool done = false;
    xcorr_status status = XCORR_OK;
    double t_submit = 0, t_done = 0, deadline = 0;
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
    double period_ms = 0;           // deadline per sample (0: windows have none)
};

// A launch of one format group being timed for the tuner.
struct Timed {
    std::string key;
    int group = 0;
    int cand = -1;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    double cmac = 0;
};

struct Launch {
    hipEvent_t done = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;   // the whole launch, for the throughput model
    double cmac = 0, est_ms = 0;
    std::vector<int64_t> tickets;
    std::vector<int32_t> sids;
    std::vector<xcorr_dump_info> info;
    std::vector<Timed> timed;
    xcorr_status status = XCORR_OK;
};

// Launch configurations tried for one mix of streams (a format group and
// the shapes of the streams admitted in it): each candidate runs kTuneRuns
// launches, then the one with the most complex MACs per second of launch
// time is kept.
constexpr int kTuneRuns = 3;
struct Tune {
    std::vector<xcorr_batch_config> cands;
    std::vector<double> cmac, ms;
    std::vector<int> runs;
    int next = 0;
    bool settled = false;
    xcorr_batch_config best{};
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

    std::map<std::string, Tune> tunes;
    std::string tune_path;          // on-disk cache of settled configurations ("" = none)

    // throughput model of a launch, est = kLaunchMs + cmac * ms_per_cmac,
    // ms_per_cmac a running average of the timed launches
    double ms_per_cmac = 0;
    double backlog_ms = 0;          // estimated time of the launches queued on the GPU

    int64_t windows_done = 0, launches = 0, batched_windows = 0, misses = 0;
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

// The format group of a plan: one persistent launch per group.
int group_of(const xcorr_plan_s* p)
{
    return p->d.format == XCORR_CI8 ? 2 : (p->n_cols % 16 == 0 ? 0 : 1);
}

// Key of a mix: the group and the sorted shapes of the admitted streams in it.
std::string mix_key(xcorr_server_t s, int group)
{
    std::vector<std::pair<int, int>> shapes;
    for (auto& kv : s->streams)
        if (kv.second.plan && group_of(kv.second.plan) == group)
            shapes.emplace_back(kv.second.desc.n_inputs, kv.second.desc.n_channels);
    std::sort(shapes.begin(), shapes.end());
    std::ostringstream o;
    o << "g" << group << "_cu" << s->n_cu;
    for (auto& sh : shapes) o << "_" << sh.first << "x" << sh.second;
    return o.str();
}

Tune& tune_for(xcorr_server_t s, const std::string& key, int group)
{
    auto it = s->tunes.find(key);
    if (it != s->tunes.end()) return it->second;
    Tune t;
    const int g1 = ((s->n_cu + 7) / 8) * 8;
    const std::vector<int> tiles = group == 0 ? std::vector<int>{kTileDma4, kTileDma8} : std::vector<int>{kTileRegs};
    for (int tile : tiles)
        for (int grid : {g1, 2 * g1})
            for (int bal : {1, 0}) t.cands.push_back(xcorr_batch_config{tile, grid, bal, 0});
    t.cmac.assign(t.cands.size(), 0);
    t.ms.assign(t.cands.size(), 0);
    t.runs.assign(t.cands.size(), 0);
    return s->tunes.emplace(key, t).first->second;
}

// Cache file: one settled configuration per line, "key tile grid balance".
void load_tunes(xcorr_server_t s)
{
    if (s->tune_path.empty()) return;
    FILE* f = std::fopen(s->tune_path.c_str(), "r");
    if (!f) return;
    char key[512];
    int tile, grid, bal;
    while (std::fscanf(f, "%511s %d %d %d", key, &tile, &grid, &bal) == 4) {
        if (tile < 0 || tile > kTileRegs || grid < 8 || grid % 8 || grid > 65536 || (bal != 0 && bal != 1)) continue;
        Tune t;
        t.settled = true;
        t.best = xcorr_batch_config{tile, grid, bal, 0};
        s->tunes[key] = t;
    }
    std::fclose(f);
}

void save_tune(xcorr_server_t s, const std::string& key, const xcorr_batch_config& c)
{
    if (s->tune_path.empty()) return;
    FILE* f = std::fopen(s->tune_path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d\n", key.c_str(), c.tile, c.grid, c.balance);
    std::fclose(f);
}

// The configuration of a group's next launch (lock held): the settled one,
// or the next candidate still being timed (cand receives its index).
xcorr_batch_config pick_config(xcorr_server_t s, const std::string& key, int group, int* cand)
{
    Tune& t = tune_for(s, key, group);
    *cand = -1;
    if (t.settled) return t.best;
    const int n = (int)t.cands.size();
    for (int k = 0; k < n; ++k) {
        const int c = (t.next + k) % n;
        if (t.runs[c] < kTuneRuns) {
            t.next = (c + 1) % n;
            *cand = c;
            return t.cands[c];
        }
    }
    return t.cands[0];
}

// A timed launch completed (lock held): record it; settle once every
// candidate has its runs.
void record_timing(xcorr_server_t s, const Timed& tm, float ms)
{
    auto it = s->tunes.find(tm.key);
    if (it == s->tunes.end() || it->second.settled || tm.cand < 0) return;
    Tune& t = it->second;
    t.cmac[tm.cand] += tm.cmac;
    t.ms[tm.cand] += ms;
    t.runs[tm.cand] += 1;
    for (int r : t.runs)
        if (r < kTuneRuns) return;
    int best = 0;
    for (size_t c = 1; c < t.cands.size(); ++c)
        if (t.cmac[c] / t.ms[c] > t.cmac[best] / t.ms[best]) best = (int)c;
    t.settled = true;
    t.best = t.cands[best];
    save_tune(s, tm.key, t.best);
}

// Enqueues one batched launch of the given windows (lock not held; the
// configuration of each group, cfgs[group], was picked with it held).
xcorr_status launch_windows(xcorr_server_t s, const std::vector<xcorr_plan_t>& plans,
                            const std::vector<Window>& ws, const std::map<int, xcorr_batch_config>& cfgs, Launch& L)
{
    std::map<int, std::vector<size_t>> groups;
    for (size_t k = 0; k < plans.size(); ++k) groups[group_of(plans[k])].push_back(k);
    L.info.assign(plans.size(), xcorr_dump_info{});
    for (auto& g : groups) {
        std::vector<xcorr_plan_t> gp;
        std::vector<const void*> in;
        std::vector<int64_t> nt;
        std::vector<void*> out;
        double cmac = 0;
        for (size_t k : g.second) {
            gp.push_back(plans[k]);
            in.push_back(ws[k].d_in);
            nt.push_back(ws[k].n_time);
            out.push_back(ws[k].d_out);
            cmac += (double)plans[k]->n_b * plans[k]->d.n_channels * (double)ws[k].n_time;
        }
        Timed* tm = nullptr;
        for (Timed& t : L.timed)
            if (t.group == g.first) tm = &t;
        if (tm) {
            tm->cmac = cmac;
            hipError_t e = hipEventCreate(&tm->t0);
            if (e == hipSuccess) e = hipEventCreate(&tm->t1);
            if (e == hipSuccess) e = hipEventRecord(tm->t0, s->stream);
            if (e != hipSuccess) return hip_fail(e, "server timing event");
        }
        std::vector<xcorr_dump_info> info;
        xcorr_status rc = run_fused_windows(s->stream, s->d_counters, cfgs.at(g.first), gp, in, nt, out, info);
        if (rc != XCORR_OK) return rc;
        if (tm) {
            hipError_t e = hipEventRecord(tm->t1, s->stream);
            if (e != hipSuccess) return hip_fail(e, "server timing event");
        }
        for (size_t j = 0; j < g.second.size(); ++j) L.info[g.second[j]] = info[j];
    }
    hipError_t e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(L.done, s->stream);
    if (e != hipSuccess) return hip_fail(e, "server event");
    return XCORR_OK;
}

// Windows one launch takes at most, and the fixed cost a launch is
// estimated at (host enqueue and the kernel's start and end).
constexpr int kMaxLaunchWindows = 96;
constexpr double kLaunchMs = 0.02;
constexpr double kCatchUpMs = 0.25;

void worker_main(xcorr_server_t s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        admit_locked(s);
        if (pending_admitted_locked(s) && (int)s->inflight.size() < s->d.max_inflight) {
            // continuous batching, earliest deadline first: the windows that
            // have arrived, of every admitted stream, in order of deadline
            // (windows without one after, in arrival order), each stream's
            // in its own order; a window joins while the launch's estimated
            // time still lets every window in it that can meet its deadline
            // meet it (the first always joins; up to kMaxLaunchWindows).  A
            // window longer than the fold bound adds chunks through its
            // plan's accumulators, and a stream whose rows are staged zero
            // padded stages into the plan's one buffer: no other window of
            // such a stream joins that launch.
            std::vector<xcorr_plan_t> plans;
            std::vector<Window> ws;
            Launch L;
            struct Cand {
                double deadline;
                int64_t ticket;
                int32_t sid;
                size_t pos;
            };
            std::vector<Cand> cands;
            for (auto& kv : s->streams) {
                Stream& st = kv.second;
                if (!st.plan) continue;
                for (size_t q = 0; q < st.pending.size() && q < (size_t)kMaxLaunchWindows; ++q)
                    cands.push_back(Cand{st.pending[q].deadline, st.pending[q].ticket, kv.first, q});
            }
            std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) {
                return a.deadline != b.deadline ? a.deadline < b.deadline : a.ticket < b.ticket;
            });
            const double now = now_ms();
            // limit: the time the launch must end by, the earliest deadline
            // of its windows that will still be met; if the most urgent
            // window is late anyway, the launch may run to twice its own
            // time (at least kCatchUpMs) to catch up on the queue
            double est = kLaunchMs, limit = std::numeric_limits<double>::infinity();
            std::map<int32_t, size_t> taken;          // windows taken from the front of each stream
            std::map<int32_t, bool> alone;
            for (const Cand& c : cands) {
                if ((int)ws.size() >= kMaxLaunchWindows) break;
                Stream& st = s->streams[c.sid];
                if (c.pos != taken[c.sid]) continue;   // an earlier window of its stream stayed out
                const Window& w = st.pending[c.pos];
                const bool solo = w.n_time > st.plan->fold_bound || st.plan->n_cols != st.plan->d.n_inputs;
                if (taken[c.sid] > 0 && (solo || alone[c.sid])) continue;
                const double e2 = est + w.cmac * s->ms_per_cmac;
                if (!ws.empty() && now + s->backlog_ms + e2 > limit) continue;
                est = e2;
                const double end = now + s->backlog_ms + est;
                if (end <= w.deadline) limit = std::min(limit, w.deadline);
                else if (ws.empty()) limit = end + std::max(est, kCatchUpMs);
                alone[c.sid] = solo;
                taken[c.sid] += 1;
                plans.push_back(st.plan);
                ws.push_back(w);
                L.tickets.push_back(w.ticket);
                L.sids.push_back(c.sid);
                L.cmac += w.cmac;
            }
            for (auto& kv : taken) {
                Stream& st = s->streams[kv.first];
                for (size_t q = 0; q < kv.second; ++q) st.pending.pop_front();
                st.inflight += (int)kv.second;
            }
            L.est_ms = est;
            s->backlog_ms += est;
            // the configuration of each format group: the tuner's
            std::map<int, xcorr_batch_config> cfgs;
            for (xcorr_plan_t p : plans) {
                const int g = group_of(p);
                if (cfgs.count(g)) continue;
                const std::string key = mix_key(s, g);
                int cand = -1;
                cfgs[g] = pick_config(s, key, g, &cand);
                if (cand >= 0) {
                    Timed tm;
                    tm.key = key;
                    tm.group = g;
                    tm.cand = cand;
                    L.timed.push_back(tm);
                }
            }
            s->launches += 1;
            s->batched_windows += (int64_t)ws.size();
            lk.unlock();
            hipError_t te = hipEventCreate(&L.t0);
            if (te == hipSuccess) te = hipEventCreate(&L.t1);
            if (te == hipSuccess) te = hipEventRecord(L.t0, s->stream);
            L.status = te != hipSuccess ? hip_fail(te, "server launch event") : launch_windows(s, plans, ws, cfgs, L);
            if (L.status == XCORR_OK && hipEventRecord(L.t1, s->stream) != hipSuccess)
                L.status = XCORR_ERR_DEVICE;
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
            float launch_ms = -1.f;
            if (L.t0 && L.t1 && L.status == XCORR_OK && hipEventElapsedTime(&launch_ms, L.t0, L.t1) != hipSuccess)
                launch_ms = -1.f;
            if (L.t0) (void)hipEventDestroy(L.t0);
            if (L.t1) (void)hipEventDestroy(L.t1);
            std::vector<float> tms(L.timed.size(), -1.f);
            for (size_t k = 0; k < L.timed.size(); ++k) {
                Timed& tm = L.timed[k];
                if (tm.t0 && tm.t1 && L.status == XCORR_OK && hipEventElapsedTime(&tms[k], tm.t0, tm.t1) != hipSuccess)
                    tms[k] = -1.f;
                if (tm.t0) (void)hipEventDestroy(tm.t0);
                if (tm.t1) (void)hipEventDestroy(tm.t1);
            }
            const double t = now_ms();
            lk.lock();
            for (size_t k = 0; k < L.timed.size(); ++k)
                if (tms[k] > 0) record_timing(s, L.timed[k], tms[k]);
            s->backlog_ms = std::max(0.0, s->backlog_ms - L.est_ms);
            if (launch_ms > kLaunchMs && L.cmac > 0) {
                const double r = (launch_ms - kLaunchMs) / L.cmac;
                s->ms_per_cmac = s->ms_per_cmac > 0 ? 0.9 * s->ms_per_cmac + 0.1 * r : r;
            }
            for (size_t k = 0; k < L.tickets.size(); ++k) {
                Ticket& tk = s->tickets[L.tickets[k]];
                tk.done = true;
                tk.status = L.status;
                tk.t_done = t;
                tk.info = L.info.empty() ? xcorr_dump_info{} : L.info[k];
                s->streams[L.sids[k]].inflight -= 1;
                if (L.status == XCORR_OK) {
                    s->misses += t > tk.deadline;
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
    if (d->tune_path) s->tune_path = d->tune_path;
    load_tunes(s);
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
    tk.deadline = it->second.period_ms > 0 ? tk.t_submit + it->second.period_ms * (double)n_time
                                           : std::numeric_limits<double>::infinity();
    if (s->first_submit < 0) s->first_submit = tk.t_submit;
    it->second.pending.push_back(Window{t, d_in, n_time, d_out, tk.deadline, tk.cmac});
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

xcorr_status xcorr_server_set_deadline(xcorr_server_t s, int32_t sid, double sample_period_s)
{
    if (!server_live(s)) return fail(XCORR_ERR_STATE, "invalid server handle");
    if (!(sample_period_s >= 0) || sample_period_s > 1e3) return fail(XCORR_ERR_ARG, "sample period out of range");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->streams.find(sid);
    if (it == s->streams.end() || it->second.closing) return fail(XCORR_ERR_ARG, "unknown or closed stream %d", sid);
    it->second.period_ms = sample_period_s * 1e3;
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
    st->deadline_misses = s->misses;
    st->mixes_tuned = 0;
    st->mixes_tuning = 0;
    for (auto& kv : s->tunes) (kv.second.settled ? st->mixes_tuned : st->mixes_tuning) += 1;
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
