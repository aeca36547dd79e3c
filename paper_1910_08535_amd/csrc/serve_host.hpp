// serve_host.hpp -- host side of the serving API (included by iga.hip, same unit).
//
// A request loop inside the library.  Requests are admitted in submission order while the
// device bytes of the requests in flight stay within the budget.  A request that the
// batched iterations take (serve_batch.hpp: every axis of at least 3p+1 elements) becomes
// a job; any other runs at once on the stream of its mesh's context (contexts cached,
// least recently used first out beyond a byte limit, bound round-robin to a pool of
// streams).  While fewer than two iterations are in flight and some job has work left,
// the loop enqueues the next iteration on a stream of its own: the descriptors of the
// iteration (one host-to-device copy), the set-up of the jobs admitted since the last
// one, then one launch per kind of job (1D, 2D, 3D per degree and output mode) over all
// jobs, the kinds side by side on streams forked from that stream and joined back.  A
// right-hand-side job runs in one iteration, a step job in one per step.
// Completion is observed from HIP events, never waited for.
#pragma once

#include <array>
#include <chrono>
#include <deque>
#include <list>
#include <unordered_map>

#include "batch.hpp"
#include "serve_batch.hpp"

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
    // requests run on contexts
    struct Item {
        uint64_t ticket;
        iga_request r;
        size_t bytes;
        hipEvent_t ev;
    };
    std::deque<Item> waiting;
    std::vector<std::deque<Item>> inflight;   // per stream, in launch order
    std::vector<hipEvent_t> events;           // free events
    // batched jobs
    struct Job {
        uint64_t ticket;
        iga_request r;
        size_t bytes;          // counted against the budget
        int R[3];              // rows (= coefficients) per axis
        int left;              // iterations still to enqueue (RHS 1, STEP nsteps)
        int k;                 // steps enqueued
        bool setup;            // tables still to expand
        double* tab;           // tables: per axis M | D [| S | F] (2D, 3D), F (1D step)
        double* work;          // step: work buffer
        int block;             // the memory block holding tab and work
        iga::Plan3D pl;        // 3D tiles
        size_t lds3;           // their LDS bytes
    };
    std::list<Job> jobs;       // admitted and unfinished, in admission order
    std::vector<std::list<Job>::iterator> fresh;   // admitted since the last iteration
    int64_t pending = 0;       // jobs with iterations still to enqueue
    struct Block {
        void* mem;
        int refs;
    };
    std::unordered_map<int, Block> blocks;
    int next_block = 0;
    struct Slot {
        hipEvent_t ev = nullptr;
        bool busy = false;
        int64_t iter = -1;
        std::vector<std::list<Job>::iterator> finishing;
        char* host = nullptr;   // pinned staging of the iteration's descriptors
        char* dev = nullptr;    // their device copy
        size_t cap = 0;
    };
    Slot slot[2];
    hipStream_t bstream = nullptr;
    // memory of batched jobs: a pool of the server's own (kept, not released), so that its
    // allocations never wait on memory that other streams freed into the device's default
    // pool (with the default pool, the real-time p99 rose from 1.3 to 5 ms after a
    // workload that had freed large buffers on other streams)
    hipMemPool_t pool = nullptr;
    // the kinds of job of an iteration (1D, 2D, 3D) run side by side on streams of their
    // own, forked from and joined back into bstream
    hipStream_t fstream[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
    const double* gen[iga::kMaxP + 1] = {};   // element-unit PG rows of (p, p+1)
    int grid2d = 0;                           // workgroups of the persistent 2D launch
    int64_t launches = 0;                     // iterations enqueued
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

// The batched iterations take a request whose mesh passes the checks of iga_create and
// whose every axis has at least 3p+1 elements (where the element-unit rows hold).
bool batchable(const iga_request& r)
{
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
    if (validate_desc(&d) != IGA_OK) return false;
    for (int a = 0; a < r.dim; ++a)
        if (r.ne[a] < iga::pg_generic_min_ne(r.p)) return false;
    return true;
}

// Doubles of a batched job's own tables: M | D per axis, and the step's S | F (2D, 3D);
// the step's source rows F when it has a source (1D).
size_t job_table_doubles(const iga_request& r)
{
    const bool step = r.kind == IGA_REQ_STEP;
    if (r.dim == 1) return step && r.sin_amp != 0.0 ? (size_t)(r.ne[0] + r.p) : 0;
    const int W = 2 * r.p + 1;
    size_t n = 0;
    for (int a = 0; a < r.dim; ++a) n += (size_t)(r.ne[a] + r.p) * (2 * W + (step ? 2 : 0));
    return n;
}

// resident bytes of a request in flight: coefficients and outputs, or coefficients and
// the step's work buffer; a batched job's tables on top
size_t request_bytes(const iga_request& r)
{
    size_t b = (r.kind == IGA_REQ_RHS ? 3 : 2) * request_points(r) * sizeof(double);
    if (batchable(r)) b += job_table_doubles(r) * sizeof(double);
    return b;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device bytes of a job's region: its tables, then the step's work buffer.
size_t job_region(const iga_server::Job& j)
{
    size_t b = up256(job_table_doubles(j.r) * sizeof(double));
    if (j.r.kind == IGA_REQ_STEP) b += up256(request_points(j.r) * sizeof(double));
    return b;
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

// ---- batched iterations -------------------------------------------------------------

void server_release_block(iga_server* s, int b)
{
    if (b < 0) return;
    auto it = s->blocks.find(b);
    if (it == s->blocks.end() || --it->second.refs > 0) return;
    // ordered after every kernel enqueued so far; the last users are complete
    (void)hipFreeAsync(it->second.mem, s->bstream);
    s->blocks.erase(it);
}

void server_finish_job(iga_server* s, std::list<iga_server::Job>::iterator j, int32_t state, int64_t launch)
{
    s->used -= j->bytes;
    if (j->left > 0) --s->pending;
    server_release_block(s, j->block);
    s->done.push_back({j->ticket, server_time(s), state, launch});
    s->jobs.erase(j);
}

// The descriptor arrays of one iteration, laid out in one buffer (256-byte aligned arrays).
struct IterLayout {
    size_t ctl, eu, eb, j1, b1, j2, j3[4], b3[4], total;
};

template <typename T>
void put(char* base, size_t off, const std::vector<T>& v)
{
    if (!v.empty()) std::memcpy(base + off, v.data(), v.size() * sizeof(T));
}

// The axis descriptor of axis a of a batched 2D/3D job (tables in tab at *off).
AxisOp job_axis(const iga_server::Job& j, int a, size_t* off)
{
    AxisOp o;
    std::memset(&o, 0, sizeof(o));
    const int W = 2 * j.r.p + 1, R = j.R[a];
    const bool step = j.r.kind == IGA_REQ_STEP;
    o.M = j.tab + *off;
    o.D = o.M + (size_t)R * W;
    // the right-hand side reads no scale or source rows: any table of R rows will do
    o.S = step ? o.D + (size_t)R * W : o.M;
    o.F = step ? o.S + R : o.M;
    o.R = o.N = R;
    o.ilo = 2 * j.r.p;
    o.ihi = (int)j.r.ne[a] - 1 - j.r.p;
    *off += (size_t)R * (2 * W + (step ? 2 : 0));
    return o;
}

// Enqueues the next iteration if a slot is free and some job has work left: set-up of the
// jobs admitted since the last iteration, then every job's next kernel.
int server_iterate(iga_server* s)
{
    using namespace iga;
    if (s->pending == 0) return IGA_OK;
    iga_server::Slot* sl = nullptr;
    for (auto& x : s->slot)
        if (!x.busy) {
            sl = &x;
            break;
        }
    if (!sl) return IGA_OK;
    // memory of the newly admitted jobs: one block
    size_t total = 0;
    int holders = 0;
    for (auto it : s->fresh) {
        const size_t b = job_region(*it);
        total += b;
        holders += b > 0;
    }
    char* base = nullptr;
    int blk = -1;
    if (total > 0) {
        void* mem = nullptr;
        if (hipMallocFromPoolAsync(&mem, total, s->pool, s->bstream) != hipSuccess) {
            (void)hipGetLastError();
            for (auto it : s->fresh) server_finish_job(s, it, IGA_JOB_FAILED, -1);
            s->fresh.clear();
            return IGA_OK;
        }
        blk = s->next_block++;
        s->blocks[blk] = {mem, holders};
        base = (char*)mem;
    }
    std::vector<ExpandUnit> eu;
    std::vector<int> eb;
    int nbe = 0;
    size_t off = 0;
    for (auto it : s->fresh) {
        iga_server::Job& j = *it;
        const iga_request& r = j.r;
        const size_t b = job_region(j);
        if (b > 0) {
            j.tab = (double*)(base + off);
            j.work = r.kind == IGA_REQ_STEP ? (double*)(base + off + up256(job_table_doubles(r) * sizeof(double)))
                                            : nullptr;
            j.block = blk;
            off += b;
        }
        const bool step = r.kind == IGA_REQ_STEP;
        size_t toff = 0;
        for (int a = 0; a < r.dim; ++a) {
            if (r.dim == 1 && !(step && r.sin_amp != 0.0)) break;
            ExpandUnit u;
            std::memset(&u, 0, sizeof(u));
            u.gen = s->gen[r.p];
            const int W = 2 * r.p + 1, R = j.R[a];
            if (r.dim == 1) {
                u.F = j.tab;
            } else {
                u.M = j.tab + toff;
                u.D = u.M + (size_t)R * W;
                if (step) {
                    u.S = u.D + (size_t)R * W;
                    u.F = u.S + R;
                    u.ones = r.sin_amp == 0.0;
                }
                toff += (size_t)R * (2 * W + (step ? 2 : 0));
            }
            u.lo = 0.0;
            u.hi = 1.0;
            u.p = r.p;
            u.nq = r.p + 1;
            u.ne = (int)r.ne[a];
            u.R = R;
            eu.push_back(u);
            eb.push_back(nbe);
            nbe += (R + kServeBlock - 1) / kServeBlock;
        }
        if (step && (r.nsteps & 1)) {   // odd: the steps start from a copy, the last lands in u
            ExpandUnit u;
            std::memset(&u, 0, sizeof(u));
            u.src = r.u;
            u.dst = j.work;
            u.n = (long long)request_points(r);
            eu.push_back(u);
            eb.push_back(nbe);
            nbe += (int)((u.n + kServeBlock - 1) / kServeBlock);
        }
        j.setup = false;
    }
    s->fresh.clear();
    // every job's next kernel
    constexpr int kTY = 16;
    std::vector<Job1D> j1;
    std::vector<int> b1;
    int nb1 = 0;
    std::vector<BatchJobDev> j2;
    int chunks = 0;
    std::vector<Job3D> j3[4];
    std::vector<int> b3[4];
    int nb3[4] = {0, 0, 0, 0};
    size_t lds3[4] = {0, 0, 0, 0};
    std::vector<std::list<iga_server::Job>::iterator> advanced;   // jobs with a kernel in this iteration
    for (auto it = s->jobs.begin(); it != s->jobs.end(); ++it) {
        iga_server::Job& j = *it;
        if (j.left == 0) continue;
        advanced.push_back(it);
        const iga_request& r = j.r;
        const bool step = r.kind == IGA_REQ_STEP;
        const double *src = r.u;
        double* dst = r.lap_out;
        if (step) {
            double* first = (r.nsteps & 1) ? j.work : r.u;
            double* second = first == r.u ? j.work : r.u;
            src = (j.k & 1) ? second : first;
            dst = (j.k & 1) ? first : second;
        }
        if (r.dim == 1) {
            Job1D d;
            std::memset(&d, 0, sizeof(d));
            d.gen = s->gen[r.p];
            d.u = src;
            d.out = dst;
            d.omass = step ? nullptr : r.mass_out;
            d.F = step && r.sin_amp != 0.0 ? j.tab : nullptr;
            d.lo = 0.0;
            d.hi = 1.0;
            d.alpha = step ? 1.0 : 0.0;
            d.beta = step ? r.dt : 1.0;
            d.gsep = step ? r.dt * r.sin_amp : 0.0;
            d.p = r.p;
            d.ne = (int)r.ne[0];
            d.step = step;
            j1.push_back(d);
            b1.push_back(nb1);
            nb1 += (j.R[0] + kServeBlock - 1) / kServeBlock;
        } else {
            ApplyArgs g;
            std::memset(&g, 0, sizeof(g));
            size_t toff = 0;
            for (int a = 0; a < r.dim; ++a) g.ax[a] = job_axis(j, a, &toff);
            g.u = src;
            g.out = dst;
            g.omass = step ? nullptr : r.mass_out;
            g.alpha = step ? 1.0 : 0.0;
            g.beta = step ? r.dt : 1.0;
            g.gsep = step ? r.dt * r.sin_amp : 0.0;
            g.garr = step ? r.dt : 0.0;
            if (r.dim == 2) {
                BatchJobDev d;
                std::memset(&d, 0, sizeof(d));
                d.g = g;
                d.p = r.p;
                d.vec = (g.ax[0].N % 2 == 0 && g.ax[0].R % 2 == 0) ? 1 : 0;
                d.tx = (g.ax[0].R + 127) / 128;
                d.ty = (g.ax[1].R + kTY - 1) / kTY;
                d.chunk0 = chunks;
                d.step = step;
                chunks += d.tx * d.ty;
                j2.push_back(d);
            } else {
                const int q = (r.p - 2) * 2 + (step ? 1 : 0);
                Job3D d;
                d.g = g;
                d.pl = j.pl;
                j3[q].push_back(d);
                b3[q].push_back(nb3[q]);
                nb3[q] += j.pl.nblk;
                lds3[q] = std::max(lds3[q], j.lds3);
            }
        }
    }
    // descriptors: one host-to-device copy
    IterLayout L;
    size_t o = 0;
    auto place = [&](size_t bytes) {
        const size_t at = o;
        o = up256(o + bytes);
        return at;
    };
    L.ctl = place(sizeof(BatchCtl));
    L.eu = place(eu.size() * sizeof(ExpandUnit));
    L.eb = place(eb.size() * sizeof(int));
    L.j1 = place(j1.size() * sizeof(Job1D));
    L.b1 = place(b1.size() * sizeof(int));
    L.j2 = place(j2.size() * sizeof(BatchJobDev));
    for (int q = 0; q < 4; ++q) {
        L.j3[q] = place(j3[q].size() * sizeof(Job3D));
        L.b3[q] = place(b3[q].size() * sizeof(int));
    }
    L.total = o;
    if (L.total > sl->cap) {
        const size_t cap = L.total + L.total / 2;
        if (sl->host) (void)hipHostFree(sl->host);
        if (sl->dev) (void)hipFreeAsync(sl->dev, s->bstream);
        sl->host = nullptr;
        sl->dev = nullptr;
        sl->cap = 0;
        IGA_HIP(hipHostMalloc((void**)&sl->host, cap, 0));
        IGA_HIP(hipMallocAsync((void**)&sl->dev, cap, s->bstream));
        sl->cap = cap;
    }
    BatchCtl ctl;
    std::memset(&ctl, 0, sizeof(ctl));
    ctl.njobs = (int)j2.size();
    ctl.total = chunks;
    std::memcpy(sl->host + L.ctl, &ctl, sizeof(ctl));
    put(sl->host, L.eu, eu);
    put(sl->host, L.eb, eb);
    put(sl->host, L.j1, j1);
    put(sl->host, L.b1, b1);
    put(sl->host, L.j2, j2);
    for (int q = 0; q < 4; ++q) {
        put(sl->host, L.j3[q], j3[q]);
        put(sl->host, L.b3[q], b3[q]);
    }
    hipStream_t st = s->bstream;
    char* dv = sl->dev;
    IGA_HIP(hipMemcpyAsync(dv, sl->host, L.total, hipMemcpyHostToDevice, st));
    if (!eu.empty())
        hipLaunchKernelGGL(serve_expand_kernel, dim3(nbe), dim3(kServeBlock), 0, st, (const ExpandUnit*)(dv + L.eu),
                           (const int*)(dv + L.eb), (int)eu.size());
    const bool has[3] = {!j1.empty(), !j2.empty(), !(j3[0].empty() && j3[1].empty() && j3[2].empty() && j3[3].empty())};
    const bool forked = (int)has[0] + (int)has[1] + (int)has[2] > 1;
    hipStream_t ks[3] = {st, st, st};
    if (forked) {
        IGA_HIP(hipEventRecord(s->fork, st));
        for (int f = 0; f < 3; ++f)
            if (has[f]) {
                ks[f] = s->fstream[f];
                IGA_HIP(hipStreamWaitEvent(ks[f], s->fork, 0));
            }
    }
    if (has[0])
        hipLaunchKernelGGL(serve1d_kernel, dim3(nb1), dim3(kServeBlock), 0, ks[0], (const Job1D*)(dv + L.j1),
                           (const int*)(dv + L.b1), (int)j1.size());
    if (has[1])
        hipLaunchKernelGGL((batch2d_kernel<kTY, true>), dim3(s->grid2d), dim3(64), 0, ks[1], (BatchCtl*)(dv + L.ctl),
                           (const BatchJobDev*)(dv + L.j2));
    for (int q = 0; q < 4; ++q) {
        if (j3[q].empty()) continue;
        const Job3D* jd = (const Job3D*)(dv + L.j3[q]);
        const int* bd = (const int*)(dv + L.b3[q]);
        const int n = (int)j3[q].size();
        hipStream_t k3 = ks[2];
        if (q == 0)
            hipLaunchKernelGGL((serve3d_kernel<2, kOut | kMass>), dim3(nb3[q]), dim3(kMaxNT3), lds3[q], k3, jd, bd, n);
        else if (q == 1)
            hipLaunchKernelGGL((serve3d_kernel<2, kOut | kScaleSrc>), dim3(nb3[q]), dim3(kMaxNT3), lds3[q], k3, jd, bd,
                               n);
        else if (q == 2)
            hipLaunchKernelGGL((serve3d_kernel<3, kOut | kMass>), dim3(nb3[q]), dim3(kMaxNT3), lds3[q], k3, jd, bd, n);
        else
            hipLaunchKernelGGL((serve3d_kernel<3, kOut | kScaleSrc>), dim3(nb3[q]), dim3(kMaxNT3), lds3[q], k3, jd, bd,
                               n);
    }
    IGA_HIP(hipGetLastError());
    if (forked)
        for (int f = 0; f < 3; ++f)
            if (has[f]) {
                IGA_HIP(hipEventRecord(s->join[f], ks[f]));
                IGA_HIP(hipStreamWaitEvent(st, s->join[f], 0));
            }
    IGA_HIP(hipEventRecord(sl->ev, st));
    // the iteration is enqueued: every job it carries has taken its next step
    for (auto it : advanced) {
        if (it->r.kind == IGA_REQ_STEP) ++it->k;
        if (--it->left == 0) {
            --s->pending;
            sl->finishing.push_back(it);
        }
    }
    sl->busy = true;
    sl->iter = s->launches++;
    return IGA_OK;
}

int server_progress(iga_server* s)
{
    // completions: events of each stream in launch order, then the iterations in order
    for (auto& q : s->inflight) {
        while (!q.empty()) {
            const hipError_t st = hipEventQuery(q.front().ev);
            if (st == hipErrorNotReady) break;
            if (st != hipSuccess) return IGA_E_DEVICE;
            server_finish(s, q.front(), IGA_JOB_DONE, -1);
            q.pop_front();
        }
    }
    for (;;) {
        iga_server::Slot* sl = nullptr;
        for (auto& x : s->slot)
            if (x.busy && (!sl || x.iter < sl->iter)) sl = &x;
        if (!sl) break;
        const hipError_t st = hipEventQuery(sl->ev);
        if (st == hipErrorNotReady) break;
        if (st != hipSuccess) return IGA_E_DEVICE;
        for (auto it : sl->finishing) server_finish_job(s, it, IGA_JOB_DONE, sl->iter);
        sl->finishing.clear();
        sl->busy = false;
    }
    // admission, in submission order
    while (!s->waiting.empty()) {
        iga_server::Item& it = s->waiting.front();
        if (s->used + it.bytes > s->budget) break;
        const iga_request& r = it.r;
        s->used += it.bytes;
        if (batchable(r) && !s->gen[r.p] && pg_generic(s->bstream, r.p, r.p + 1, &s->gen[r.p]) != IGA_OK) {
            (void)hipGetLastError();
            server_finish(s, it, IGA_JOB_FAILED, -1);   // the element-unit rows could not be built
        } else if (batchable(r)) {
            iga_server::Job j;
            std::memset(&j.pl, 0, sizeof(j.pl));
            j.ticket = it.ticket;
            j.r = r;
            j.bytes = it.bytes;
            for (int a = 0; a < 3; ++a) j.R[a] = a < r.dim ? (int)(r.ne[a] + r.p) : 1;
            j.left = r.kind == IGA_REQ_RHS ? 1 : r.nsteps;
            j.k = 0;
            j.setup = true;
            j.tab = nullptr;
            j.work = nullptr;
            j.block = -1;
            j.lds3 = 0;
            if (r.dim == 3) {
                int nt = 0;
                j.pl = plan_3d_rows(r.p, j.R[0], j.R[1], j.R[2], 0, 0, 0, &nt, &j.lds3);
            }
            s->jobs.push_back(j);
            s->fresh.push_back(std::prev(s->jobs.end()));
            ++s->pending;
        } else {
            it.ev = nullptr;
            if (server_launch(s, it) != IGA_OK) {
                (void)hipGetLastError();
                server_finish(s, it, IGA_JOB_FAILED, -1);
            }
        }
        s->peak = std::max(s->peak, s->used);
        s->waiting.pop_front();
    }
    // iterations: while a slot is free and some job has work left
    while (s->pending > 0) {
        const int64_t before = s->launches;
        IGA_TRY(server_iterate(s));
        if (s->launches == before) break;
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
    ok = ok && hipStreamCreateWithFlags(&s->bstream, hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        int dev = 0;
        hipMemPoolProps props;
        std::memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        ok = hipGetDevice(&dev) == hipSuccess;
        props.location.id = dev;
        ok = ok && hipMemPoolCreate(&s->pool, &props) == hipSuccess;
        uint64_t keep = UINT64_MAX;
        ok = ok && hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess;
    }
    for (auto& sl : s->slot) ok = ok && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&s->fork, hipEventDisableTiming) == hipSuccess;
    for (int f = 0; f < 3; ++f)
        ok = ok && hipStreamCreateWithFlags(&s->fstream[f], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&s->join[f], hipEventDisableTiming) == hipSuccess;
    if (ok) {   // the persistent 2D launch fills the chip once
        int dev = 0, ncu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, iga::batch2d_kernel<16, true>, 64, 0) != hipSuccess) {
            (void)hipGetLastError();
            ncu = 256;
            per = 4;
        }
        s->grid2d = std::max(8, ncu * std::max(per, 1));
    }
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
    for (int f = 0; f < 3; ++f)
        if (s->fstream[f]) (void)hipStreamSynchronize(s->fstream[f]);
    if (s->bstream) (void)hipStreamSynchronize(s->bstream);
    for (auto& kv : s->cache) iga_destroy(kv.second.c);
    for (auto& q : s->inflight)
        for (auto& it : q)
            if (it.ev) (void)hipEventDestroy(it.ev);
    for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
    for (auto& kv : s->blocks) (void)hipFreeAsync(kv.second.mem, s->bstream);
    for (auto& sl : s->slot) {
        if (sl.dev) (void)hipFreeAsync(sl.dev, s->bstream);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    }
    if (s->bstream) (void)hipStreamSynchronize(s->bstream);
    for (auto& sl : s->slot)
        if (sl.host) (void)hipHostFree(sl.host);
    if (s->pool) (void)hipMemPoolDestroy(s->pool);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->bstream) (void)hipStreamDestroy(s->bstream);
    for (int f = 0; f < 3; ++f) {
        if (s->fstream[f]) (void)hipStreamDestroy(s->fstream[f]);
        if (s->join[f]) (void)hipEventDestroy(s->join[f]);
    }
    if (s->fork) (void)hipEventDestroy(s->fork);
    delete s;
    return IGA_OK;
}

}  // extern "C"
