// serve_host.hpp -- host side of the serving API (included by iga.hip, same unit).
//
// A request loop inside the library: requests are admitted in submission order while
// the device bytes of the requests in flight stay within the budget.  Each admitted
// request runs at once on the stream of its mesh's context (contexts are cached, least
// recently used first out beyond a byte limit, and bound round-robin to a pool of
// streams); 2D RHS requests instead join the queue of a persistent batch launch, and one
// launch takes every queued 2D RHS request whenever no launch is running (continuous
// batching).  Completion is observed from HIP events, never waited for.
#pragma once

#include <array>
#include <chrono>
#include <deque>
#include <list>
#include <unordered_map>

struct iga_server {
    std::vector<hipStream_t> streams;
    size_t budget = 0, used = 0, peak = 0;
    size_t cache_limit = 0, cache_bytes = 0;
    int next_stream = 0;
    struct Ctx {
        iga_ctx* c;
        int stream;
        std::list<std::array<int64_t, 5>>::iterator lru;
        size_t bytes;   // device bytes of the context counted in cache_bytes
    };
    struct KeyHash {
        size_t operator()(const std::array<int64_t, 5>& k) const
        {
            size_t h = 1469598103934665603ull;
            for (int64_t v : k) h = (h ^ (size_t)v) * 1099511628211ull;
            return h;
        }
    };
    std::unordered_map<std::array<int64_t, 5>, Ctx, KeyHash> cache;
    std::list<std::array<int64_t, 5>> lru;   // front = least recently used
    // requests
    struct Item {
        uint64_t ticket;
        iga_request r;
        size_t bytes;
        hipEvent_t ev;
    };
    std::deque<Item> waiting;
    std::vector<std::deque<Item>> inflight;   // per stream, in launch order
    iga_batch* batch = nullptr;
    hipStream_t batch_stream = nullptr;
    hipEvent_t batch_ev = nullptr;
    std::vector<Item> batch_queued, batch_running;
    int64_t launches = 0;
    std::vector<hipEvent_t> events;   // free events
    struct Done {
        uint64_t ticket;
        double t;
        int32_t state;
        int64_t launch;
    };
    std::deque<Done> done;
    uint64_t next_ticket = 1;
    std::chrono::steady_clock::time_point t0;
};

namespace {

size_t request_points(const iga_request& r)
{
    size_t n = 1;
    for (int a = 0; a < r.dim; ++a) n *= (size_t)(r.ne[a] + r.p);
    return n;
}

// resident bytes of a request in flight: coefficients and outputs, or coefficients and
// the step's work buffer
size_t request_bytes(const iga_request& r)
{
    return (r.kind == IGA_REQ_RHS ? 3 : 2) * request_points(r) * sizeof(double);
}

double server_time(const iga_server* s)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

int server_event(iga_server* s, hipEvent_t* ev)
{
    if (!s->events.empty()) {
        *ev = s->events.back();
        s->events.pop_back();
        return IGA_OK;
    }
    IGA_HIP(hipEventCreateWithFlags(ev, hipEventDisableTiming));
    return IGA_OK;
}

// Evicts least recently used contexts while the cached contexts' device bytes (tables,
// scratch such as the explicit step's work buffer) exceed the limit; frees are ordered
// after each context's work.  The most recently used context always stays.
void server_evict(iga_server* s)
{
    while (s->cache_bytes > s->cache_limit && s->lru.size() > 1) {
        const auto old = s->lru.front();
        auto oi = s->cache.find(old);
        s->cache_bytes -= oi->second.bytes;
        iga_destroy(oi->second.c);
        s->cache.erase(oi);
        s->lru.pop_front();
    }
}

int server_ctx(iga_server* s, const iga_request& r, iga_server::Ctx** out)
{
    const std::array<int64_t, 5> key = {r.dim, r.p, r.ne[0], r.dim > 1 ? r.ne[1] : 1,
                                        r.dim > 2 ? r.ne[2] : 1};
    auto it = s->cache.find(key);
    if (it != s->cache.end()) {
        s->lru.splice(s->lru.end(), s->lru, it->second.lru);
        *out = &it->second;
        return IGA_OK;
    }
    iga_mesh_desc d;
    std::memset(&d, 0, sizeof(d));
    d.dim = r.dim;
    d.p = r.p;
    for (int a = 0; a < 3; ++a) {
        d.ne[a] = a < r.dim ? r.ne[a] : 1;
        d.lo[a] = 0.0;
        d.hi[a] = 1.0;
        d.nq[a] = r.p + 1;
    }
    d.spans = IGA_SPANS_SUPPORT;
    const int k = s->next_stream;
    s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
    iga_ctx* c = nullptr;
    IGA_TRY(iga_create(&d, s->streams[k], &c));
    s->lru.push_back(key);
    auto& e = s->cache[key];
    e = {c, k, std::prev(s->lru.end()), ctx_device_bytes(c)};
    s->cache_bytes += e.bytes;
    server_evict(s);
    *out = &s->cache.find(key)->second;
    return IGA_OK;
}

void server_finish(iga_server* s, const iga_server::Item& it, int32_t state, int64_t launch)
{
    s->used -= it.bytes;
    if (it.ev) s->events.push_back(it.ev);
    s->done.push_back({it.ticket, server_time(s), state, launch});
}

int server_launch(iga_server* s, iga_server::Item& it)
{
    const iga_request& r = it.r;
    iga_server::Ctx* e = nullptr;
    IGA_TRY(server_ctx(s, r, &e));
    if (r.kind == IGA_REQ_RHS) {
        IGA_TRY(iga_apply(e->c, IGA_PG, r.u, r.mass_out, r.lap_out));
    } else {
        iga_source f = {nullptr, r.sin_amp};
        IGA_TRY(iga_explicit_step(e->c, r.u, r.dt, &f, r.nsteps));
    }
    IGA_TRY(server_event(s, &it.ev));
    IGA_HIP(hipEventRecord(it.ev, s->streams[e->stream]));
    s->inflight[e->stream].push_back(it);
    // the call may have grown the context's scratch (the step's work buffer)
    const size_t now = ctx_device_bytes(e->c);
    s->cache_bytes += now - e->bytes;
    e->bytes = now;
    server_evict(s);
    return IGA_OK;
}

int server_progress(iga_server* s)
{
    // completions: events of each stream in launch order, and the batch launch
    for (auto& q : s->inflight) {
        while (!q.empty()) {
            const hipError_t st = hipEventQuery(q.front().ev);
            if (st == hipErrorNotReady) break;
            if (st != hipSuccess) return IGA_E_DEVICE;
            server_finish(s, q.front(), IGA_JOB_DONE, -1);
            q.pop_front();
        }
    }
    if (!s->batch_running.empty()) {
        const hipError_t st = hipEventQuery(s->batch_ev);
        if (st == hipSuccess) {
            for (auto& it : s->batch_running) {
                it.ev = nullptr;
                server_finish(s, it, IGA_JOB_DONE, s->launches - 1);
            }
            s->batch_running.clear();
            IGA_TRY(iga_batch_wait(s->batch));   // retires the launch (it is done)
        } else if (st != hipErrorNotReady) {
            return IGA_E_DEVICE;
        }
    }
    // admission, in submission order
    while (!s->waiting.empty()) {
        iga_server::Item& it = s->waiting.front();
        if (s->used + it.bytes > s->budget) break;
        const iga_request& r = it.r;
        if (r.kind == IGA_REQ_RHS && r.dim == 2) {
            iga_job j;
            j.p = r.p;
            j.ne[0] = r.ne[0];
            j.ne[1] = r.ne[1];
            j.u = r.u;
            j.mass_out = r.mass_out;
            j.lap_out = r.lap_out;
            uint64_t t = 0;
            const int rc = iga_batch_submit(s->batch, &j, 1, &t);
            if (rc == IGA_E_AGAIN) break;
            it.ev = nullptr;
            s->used += it.bytes;
            if (rc != IGA_OK) {
                server_finish(s, it, IGA_JOB_FAILED, -1);
            } else {
                s->batch_queued.push_back(it);
            }
        } else {
            s->used += it.bytes;
            it.ev = nullptr;
            if (server_launch(s, it) != IGA_OK) {
                (void)hipGetLastError();
                server_finish(s, it, IGA_JOB_FAILED, -1);
            }
        }
        s->peak = std::max(s->peak, s->used);
        s->waiting.pop_front();
    }
    // a batch launch takes every queued 2D RHS request when none is running
    if (s->batch_running.empty() && !s->batch_queued.empty()) {
        const int rc = iga_batch_flush(s->batch);
        if (rc != IGA_OK) {
            for (auto& it : s->batch_queued) server_finish(s, it, IGA_JOB_FAILED, -1);
            s->batch_queued.clear();
            return IGA_OK;
        }
        IGA_HIP(hipEventRecord(s->batch_ev, s->batch_stream));
        s->batch_running.swap(s->batch_queued);
        ++s->launches;
    }
    return IGA_OK;
}

}  // namespace

extern "C" {

int iga_server_create(int32_t nstreams, size_t mem_budget_bytes, size_t cache_bytes, iga_server** out)
{
    if (!out || nstreams < 1 || nstreams > 64 || mem_budget_bytes == 0) return IGA_E_INVAL;
    *out = nullptr;
    iga_server* s = new (std::nothrow) iga_server;
    if (!s) return IGA_E_NOMEM;
    s->budget = mem_budget_bytes;
    s->cache_limit = cache_bytes;
    s->t0 = std::chrono::steady_clock::now();
    bool ok = true;
    for (int k = 0; k < nstreams && ok; ++k) {
        hipStream_t st = nullptr;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) s->streams.push_back(st);
    }
    s->inflight.resize(s->streams.size());
    ok = ok && hipStreamCreateWithFlags(&s->batch_stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&s->batch_ev, hipEventDisableTiming) == hipSuccess &&
         iga_batch_create(s->batch_stream, 0, 1 << 16, &s->batch) == IGA_OK;
    if (!ok) {
        (void)hipGetLastError();
        iga_server_destroy(s);
        return IGA_E_NOMEM;
    }
    *out = s;
    return IGA_OK;
}

int iga_server_submit(iga_server* s, const iga_request* reqs, int32_t n, uint64_t* tickets)
{
    if (!s || !reqs || !tickets || n < 0) return IGA_E_INVAL;
    for (int32_t k = 0; k < n; ++k) {   // all or nothing
        const iga_request& r = reqs[k];
        if (r.kind != IGA_REQ_RHS && r.kind != IGA_REQ_STEP) return IGA_E_INVAL;
        if (r.dim < 1 || r.dim > 3 || r.p < 2 || r.p > iga::kMaxP) return IGA_E_UNSUPPORTED;
        for (int a = 0; a < r.dim; ++a)
            if (r.ne[a] < 1 || r.ne[a] > (1 << 28)) return IGA_E_INVAL;
        if (!r.u) return IGA_E_INVAL;
        if (r.kind == IGA_REQ_RHS && (!r.mass_out || !r.lap_out || r.mass_out == r.lap_out))
            return IGA_E_INVAL;
        if (r.kind == IGA_REQ_STEP && (r.nsteps < 1 || !std::isfinite(r.dt) || !std::isfinite(r.sin_amp)))
            return IGA_E_INVAL;
        if (request_bytes(r) > s->budget) return IGA_E_NOMEM;
    }
    for (int32_t k = 0; k < n; ++k) {
        iga_server::Item it;
        it.ticket = s->next_ticket++;
        it.r = reqs[k];
        it.bytes = request_bytes(reqs[k]);
        it.ev = nullptr;
        s->waiting.push_back(it);
        tickets[k] = it.ticket;
    }
    return server_progress(s);
}

int iga_server_progress(iga_server* s, uint64_t* done, double* done_time, int32_t* done_state,
                        int64_t* done_launch, int32_t cap, int32_t* ndone)
{
    if (!s || !ndone || cap < 0 || (cap > 0 && (!done || !done_time || !done_state))) return IGA_E_INVAL;
    IGA_TRY(server_progress(s));
    int32_t m = 0;
    while (m < cap && !s->done.empty()) {
        const auto& d = s->done.front();
        done[m] = d.ticket;
        done_time[m] = d.t;
        done_state[m] = d.state;
        if (done_launch) done_launch[m] = d.launch;
        s->done.pop_front();
        ++m;
    }
    *ndone = m;
    return IGA_OK;
}

int iga_server_stats(const iga_server* s, size_t* used, size_t* peak, int64_t* batch_launches, double* now)
{
    if (!s) return IGA_E_INVAL;
    if (used) *used = s->used;
    if (peak) *peak = s->peak;
    if (batch_launches) *batch_launches = s->launches;
    if (now) *now = server_time(s);
    return IGA_OK;
}

int iga_server_cache_stats(const iga_server* s, size_t* cache_bytes, int64_t* contexts)
{
    if (!s) return IGA_E_INVAL;
    if (cache_bytes) *cache_bytes = s->cache_bytes;
    if (contexts) *contexts = (int64_t)s->cache.size();
    return IGA_OK;
}

int iga_server_destroy(iga_server* s)
{
    if (!s) return IGA_E_INVAL;
    for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
    if (s->batch_stream) (void)hipStreamSynchronize(s->batch_stream);
    if (s->batch) iga_batch_destroy(s->batch);
    for (auto& kv : s->cache) iga_destroy(kv.second.c);
    for (auto& q : s->inflight)
        for (auto& it : q)
            if (it.ev) (void)hipEventDestroy(it.ev);
    for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
    if (s->batch_ev) (void)hipEventDestroy(s->batch_ev);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->batch_stream) (void)hipStreamDestroy(s->batch_stream);
    delete s;
    return IGA_OK;
}

}  // extern "C"
