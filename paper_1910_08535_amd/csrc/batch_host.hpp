// batch_host.hpp -- host side of the batch API (included by iga.hip, same unit).
#pragma once

#include <map>
#include <set>
#include <tuple>

#include "batch.hpp"

struct iga_batch {
    hipStream_t stream = nullptr;
    size_t budget = 0;
    int max_jobs = 0;
    int ty = 8;   // chunk rows of the 2D kernel (autotuned)
    std::map<std::tuple<int, int64_t, int64_t>, iga_ctx*> meshes;   // (p, nx, ny) -> tables
    struct Item {
        uint64_t ticket;
        iga_job job;
        size_t bytes;
    };
    std::vector<Item> queued;
    size_t queued_bytes = 0;
    // the launch in flight
    std::vector<uint64_t> running;    // tickets by slot
    size_t running_bytes = 0;
    bool in_flight = false;
    uint64_t next_ticket = 1;
    std::set<uint64_t> failed;
    // device state
    iga::BatchJobDev* jobs_host = nullptr;   // pinned staging
    iga::BatchJobDev* jobs_dev = nullptr;
    iga::BatchCtl* ctl_host = nullptr;       // pinned staging
    iga::BatchCtl* ctl_dev = nullptr;
    hipEvent_t ev = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_ty = 0;
};

namespace {

size_t job_bytes(const iga_job& j)
{
    const size_t n = (size_t)(j.ne[0] + j.p) * (size_t)(j.ne[1] + j.p);
    return 3 * n * sizeof(double);
}

int batch_mesh(iga_batch* b, int p, int64_t nx, int64_t ny, iga_ctx** out)
{
    const auto key = std::make_tuple(p, nx, ny);
    auto it = b->meshes.find(key);
    if (it != b->meshes.end()) {
        *out = it->second;
        return IGA_OK;
    }
    iga_mesh_desc d;
    std::memset(&d, 0, sizeof(d));
    d.dim = 2;
    d.p = p;
    d.ne[0] = nx;
    d.ne[1] = ny;
    d.ne[2] = 1;
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = 0.0;
        d.hi[a] = 1.0;
        d.nq[a] = p + 1;
    }
    d.spans = IGA_SPANS_SUPPORT;
    iga_ctx* c = nullptr;
    IGA_TRY(iga_create(&d, b->stream, &c));
    b->meshes[key] = c;
    *out = c;
    return IGA_OK;
}

template <int TY>
int batch_grid()
{
    static int grid = 0;
    if (grid == 0) {
        int dev = 0, ncu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, iga::batch2d_kernel<TY, false>, 64, 0) !=
                hipSuccess) {
            (void)hipGetLastError();
            ncu = 256;
            per = 8;
        }
        grid = std::max(8, ncu * std::max(per, 1));
    }
    return grid;
}

template <int TY>
void batch_enqueue(iga_batch* b, hipStream_t s)
{
    hipLaunchKernelGGL(iga::batch_reset_kernel, dim3(1), dim3(64), 0, s, b->ctl_dev);
    hipLaunchKernelGGL((iga::batch2d_kernel<TY, false>), dim3(batch_grid<TY>()), dim3(64), 0, s, b->ctl_dev,
                       (const iga::BatchJobDev*)b->jobs_dev);
}

// The graph of one launch: counter reset + persistent kernel.  Its arguments are fixed
// device pointers (the job list and its size are read from device memory), so it is
// captured once per chunk height and replayed by every flush.
int batch_graph(iga_batch* b)
{
    if (b->gexec && b->graph_ty == b->ty) return IGA_OK;
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    hipStream_t cap = nullptr;
    IGA_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (b->ty == 4)
            batch_enqueue<4>(b, cap);
        else if (b->ty == 16)
            batch_enqueue<16>(b, cap);
        else
            batch_enqueue<8>(b, cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cap, &g);
        if (e == hipSuccess) {
            e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cap);
    IGA_HIP(e);
    b->graph_ty = b->ty;
    return IGA_OK;
}

// Job list of the first n queued jobs into the pinned staging buffers; returns the
// number of chunks.
int batch_fill(iga_batch* b, size_t n, int* total)
{
    int chunk = 0;
    for (size_t k = 0; k < n; ++k) {
        const iga_job& j = b->queued[k].job;
        iga_ctx* c = nullptr;
        IGA_TRY(batch_mesh(b, j.p, j.ne[0], j.ne[1], &c));
        iga::BatchJobDev& d = b->jobs_host[k];
        std::memset(&d, 0, sizeof(d));
        d.g = make_args(c, IGA_PG, false, false);
        d.g.u = j.u;
        d.g.out = j.lap_out;
        d.g.omass = j.mass_out;
        d.g.alpha = 0.0;
        d.g.beta = 1.0;
        d.p = j.p;
        d.vec = (d.g.ax[0].N % 2 == 0 && d.g.ax[0].R % 2 == 0) ? 1 : 0;
        d.tx = (d.g.ax[0].R + 127) / 128;
        d.ty = (d.g.ax[1].R + b->ty - 1) / b->ty;
        d.chunk0 = chunk;
        chunk += d.tx * d.ty;
    }
    *total = chunk;
    return IGA_OK;
}

// The job list of a launch to the device (the graph reads it from there).
int batch_upload(iga_batch* b, size_t n, int total)
{
    std::memset(b->ctl_host, 0, sizeof(iga::BatchCtl));
    b->ctl_host->njobs = (int)n;
    b->ctl_host->total = total;
    IGA_HIP(hipMemcpyAsync(b->jobs_dev, b->jobs_host, n * sizeof(iga::BatchJobDev),
                           hipMemcpyHostToDevice, b->stream));
    IGA_HIP(hipMemcpyAsync(b->ctl_dev, b->ctl_host, sizeof(iga::BatchCtl), hipMemcpyHostToDevice,
                           b->stream));
    return IGA_OK;
}

int batch_launch_prepared(iga_batch* b, size_t n, int total)
{
    IGA_TRY(batch_upload(b, n, total));
    IGA_TRY(batch_graph(b));
    IGA_HIP(hipGraphLaunch(b->gexec, b->stream));
    IGA_HIP(hipEventRecord(b->ev, b->stream));
    return IGA_OK;
}

void batch_retire(iga_batch* b)
{
    b->running.clear();
    b->running_bytes = 0;
    b->in_flight = false;
}

int batch_sync(iga_batch* b)
{
    if (!b->in_flight) return IGA_OK;
    IGA_HIP(hipEventSynchronize(b->ev));
    batch_retire(b);
    return IGA_OK;
}

}  // namespace

extern "C" {

int iga_batch_create(void* hip_stream, size_t mem_budget_bytes, int32_t max_jobs, iga_batch** out)
{
    if (!out || max_jobs < 1 || max_jobs > (1 << 20)) return IGA_E_INVAL;
    *out = nullptr;
    iga_batch* b = new (std::nothrow) iga_batch;
    if (!b) return IGA_E_NOMEM;
    b->stream = (hipStream_t)hip_stream;
    b->budget = mem_budget_bytes;
    b->max_jobs = max_jobs;
    bool ok = hipHostMalloc((void**)&b->jobs_host, sizeof(iga::BatchJobDev) * max_jobs, 0) == hipSuccess &&
              hipHostMalloc((void**)&b->ctl_host, sizeof(iga::BatchCtl), 0) == hipSuccess &&
              hipMalloc((void**)&b->jobs_dev, sizeof(iga::BatchJobDev) * max_jobs) == hipSuccess &&
              hipMalloc((void**)&b->ctl_dev, sizeof(iga::BatchCtl)) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        iga_batch_destroy(b);
        return IGA_E_NOMEM;
    }
    *out = b;
    return IGA_OK;
}

int iga_batch_submit(iga_batch* b, const iga_job* jobs, int32_t njobs, uint64_t* tickets)
{
    if (!b || !jobs || !tickets || njobs < 0) return IGA_E_INVAL;
    size_t bytes = 0;
    for (int32_t k = 0; k < njobs; ++k) {
        const iga_job& j = jobs[k];
        if (j.p < 2 || j.p > iga::kMaxP) return IGA_E_UNSUPPORTED;
        if (j.ne[0] < 1 || j.ne[1] < 1 || !j.u || !j.mass_out || !j.lap_out) return IGA_E_INVAL;
        if ((size_t)(j.ne[0] + j.p) * (size_t)(j.ne[1] + j.p) >= ((size_t)1 << 28)) return IGA_E_INVAL;
        if (j.mass_out == j.lap_out || (const double*)j.mass_out == j.u || (const double*)j.lap_out == j.u)
            return IGA_E_INVAL;
        bytes += job_bytes(j);
    }
    if (b->queued.size() + (size_t)njobs > (size_t)b->max_jobs) return IGA_E_AGAIN;
    if (b->budget && b->queued_bytes + b->running_bytes + bytes > b->budget) return IGA_E_AGAIN;
    for (int32_t k = 0; k < njobs; ++k) {
        const uint64_t t = b->next_ticket++;
        b->queued.push_back({t, jobs[k], job_bytes(jobs[k])});
        tickets[k] = t;
    }
    b->queued_bytes += bytes;
    return IGA_OK;
}

int iga_batch_flush(iga_batch* b)
{
    if (!b) return IGA_E_INVAL;
    IGA_TRY(batch_sync(b));
    if (b->queued.empty()) return IGA_OK;
    const size_t n = std::min(b->queued.size(), (size_t)b->max_jobs);
    int total = 0;
    const int rc = batch_fill(b, n, &total);
    if (rc != IGA_OK) {   // a mesh could not be set up: its jobs fail, the rest wait
        for (size_t k = 0; k < n; ++k) b->failed.insert(b->queued[k].ticket);
        for (size_t k = 0; k < n; ++k) b->queued_bytes -= b->queued[k].bytes;
        b->queued.erase(b->queued.begin(), b->queued.begin() + n);
        return rc;
    }
    IGA_TRY(batch_launch_prepared(b, n, total));
    for (size_t k = 0; k < n; ++k) {
        b->running.push_back(b->queued[k].ticket);
        b->running_bytes += b->queued[k].bytes;
        b->queued_bytes -= b->queued[k].bytes;
    }
    b->queued.erase(b->queued.begin(), b->queued.begin() + n);
    b->in_flight = true;
    return IGA_OK;
}

int iga_batch_poll(iga_batch* b, uint64_t ticket, int32_t* state)
{
    if (!b || !state || ticket == 0 || ticket >= b->next_ticket) return IGA_E_INVAL;
    if (b->failed.count(ticket)) {
        *state = IGA_JOB_FAILED;
        return IGA_OK;
    }
    for (const auto& it : b->queued)
        if (it.ticket == ticket) {
            *state = IGA_JOB_QUEUED;
            return IGA_OK;
        }
    for (size_t k = 0; k < b->running.size(); ++k)
        if (b->running[k] == ticket) {
            const hipError_t q = hipEventQuery(b->ev);
            if (q == hipSuccess) {
                batch_retire(b);
                *state = IGA_JOB_DONE;
            } else if (q == hipErrorNotReady) {
                *state = IGA_JOB_RUNNING;
            } else {
                return IGA_E_DEVICE;
            }
            return IGA_OK;
        }
    *state = IGA_JOB_DONE;   // an earlier launch, already retired
    return IGA_OK;
}

int iga_batch_wait(iga_batch* b)
{
    if (!b) return IGA_E_INVAL;
    return batch_sync(b);
}

int iga_batch_autotune(iga_batch* b, int32_t reps, int32_t* best_rows, float* best_ms)
{
    if (!b || reps < 1) return IGA_E_INVAL;
    IGA_TRY(batch_sync(b));
    if (b->queued.empty()) return IGA_E_INVAL;
    const size_t n = std::min(b->queued.size(), (size_t)b->max_jobs);
    hipEvent_t e0, e1;
    IGA_HIP(hipEventCreate(&e0));
    IGA_HIP(hipEventCreate(&e1));
    const int cand[3] = {4, 8, 16};
    float best = -1.0f;
    int best_ty = b->ty;
    int rc = IGA_OK;
    for (int ci = 0; ci < 3 && rc == IGA_OK; ++ci) {
        b->ty = cand[ci];
        int total = 0;
        rc = batch_fill(b, n, &total);
        if (rc != IGA_OK) break;
        rc = batch_launch_prepared(b, n, total);   // warm-up and graph capture
        if (rc != IGA_OK) break;
        // the job list is on the device and the graph resets the claim counter: only the
        // launches themselves are timed
        (void)hipEventRecord(e0, b->stream);
        for (int r = 0; r < reps && rc == IGA_OK; ++r)
            if (hipGraphLaunch(b->gexec, b->stream) != hipSuccess) rc = IGA_E_DEVICE;
        (void)hipEventRecord(e1, b->stream);
        if (hipEventSynchronize(e1) != hipSuccess) rc = IGA_E_DEVICE;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rc == IGA_OK && (best < 0.0f || ms < best)) {
            best = ms;
            best_ty = cand[ci];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->ty = best_ty;
    if (best_rows) *best_rows = best_ty;
    if (best_ms) *best_ms = best / (float)reps;
    return rc;
}

int iga_batch_destroy(iga_batch* b)
{
    if (!b) return IGA_E_INVAL;
    if (b->in_flight && b->ev) (void)hipEventSynchronize(b->ev);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    for (auto& kv : b->meshes) iga_destroy(kv.second);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->jobs_dev) (void)hipFree(b->jobs_dev);
    if (b->ctl_dev) (void)hipFree(b->ctl_dev);
    if (b->jobs_host) (void)hipHostFree(b->jobs_host);
    if (b->ctl_host) (void)hipHostFree(b->ctl_host);
    delete b;
    return IGA_OK;
}

}  // extern "C"
