// batch.hpp -- many independent 2D problems in one persistent launch.
//
// Every job is a fused Petrov-Galerkin apply (mass and Laplacian rows) of its own
// tensor-product space (its own p, element counts and band tables).  Its rows are cut
// into the chunks of the 2D kernel (128 columns x TY rows); the chunks of all jobs are
// numbered consecutively and cut into eight contiguous ranges, one per XCD.  Each wave of
// the persistent grid claims the next chunk of its own XCD's range from that range's
// counter, then, once it is drained, helps the other ranges in turn.  Neighbouring
// chunks share halo rows and the 128-byte lines at the strip edges; claimed on one XCD at
// about the same time, those come from its L2 instead of HBM (with one device-wide
// counter the halos cost a third more read traffic).  The jobs of a launch complete
// together with the launch: on this GPU a device-wide release (to publish one job early)
// writes back a whole L2 of an XCD, far too dear to pay per chunk.
#pragma once

#include "apply.hpp"
#include "common.hpp"

namespace iga {

struct BatchJobDev {
    ApplyArgs g;   // band tables, u, out (Laplacian rows), omass (mass rows)
    int p;         // 2 or 3
    int vec;       // rows of even length: 128-bit row accesses
    int tx, ty;    // strips and row chunks of the job
    int chunk0;    // first chunk number of the job in this launch
    int step;      // a lumped explicit step (scaled rows and source into out) instead of
                   // the mass and Laplacian rows (kernels instantiated with STEPS only)
};

constexpr int kXcds = 8;   // XCDs of the chip; workgroup b runs on XCD b mod 8

struct BatchCtl {
    int njobs;
    int total;                   // chunks over all jobs
    int pad[30];
    unsigned counter[kXcds][32];  // next claim in each XCD's range, one 128-byte line each
};

// Resets the claim counters of a launch.
__global__ void batch_reset_kernel(BatchCtl* ctl)
{
    if (blockIdx.x == 0 && threadIdx.x < kXcds) ctl->counter[threadIdx.x][0] = 0u;
}

template <int TY, bool STEPS>
__global__ __launch_bounds__(64) void batch2d_kernel(BatchCtl* ctl, const BatchJobDev* __restrict__ jobs)
{
    constexpr int LDS = Chunk2D<3, TY>::LDS > Chunk2D<2, TY>::LDS ? Chunk2D<3, TY>::LDS
                                                                 : Chunk2D<2, TY>::LDS;
    __shared__ __attribute__((aligned(16))) double lds[LDS];
    const int njobs = ctl->njobs, total = ctl->total;
    const int xcd = (int)(blockIdx.x & (kXcds - 1));
    for (int h = 0; h < kXcds; ++h) {
        const int k = (xcd + h) & (kXcds - 1);
        const int r0 = (int)((long long)total * k / kXcds);
        const int r1 = (int)((long long)total * (k + 1) / kXcds);
        for (;;) {
            unsigned c = 0;
            if (threadIdx.x == 0) c = atomicAdd(&ctl->counter[k][0], 1u);
            c = __builtin_amdgcn_readfirstlane(c);
            if ((int)c >= r1 - r0) break;
            c += (unsigned)r0;
            // the job whose chunk range holds c (jobs are sorted by chunk0)
            int lo = 0, hi = njobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].chunk0 <= (int)c)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            // a private copy: the kernel stores to global memory, so fields read through a
            // pointer would be re-read after every store
            const BatchJobDev J = jobs[lo];
            const int local = (int)c - J.chunk0;
            const int bx = local % J.tx, by = local / J.tx;
            if (STEPS && J.step) {
                constexpr int M = kOut | kScaleSrc;
                if (J.p == 2) {
                    if (J.vec)
                        apply2d_chunk<2, TY, M, true>(J.g, bx, by, lds);
                    else
                        apply2d_chunk<2, TY, M, false>(J.g, bx, by, lds);
                } else {
                    if (J.vec)
                        apply2d_chunk<3, TY, M, true>(J.g, bx, by, lds);
                    else
                        apply2d_chunk<3, TY, M, false>(J.g, bx, by, lds);
                }
            } else if (J.p == 2) {
                if (J.vec)
                    apply2d_chunk<2, TY, kOut | kMass, true>(J.g, bx, by, lds);
                else
                    apply2d_chunk<2, TY, kOut | kMass, false>(J.g, bx, by, lds);
            } else {
                if (J.vec)
                    apply2d_chunk<3, TY, kOut | kMass, true>(J.g, bx, by, lds);
                else
                    apply2d_chunk<3, TY, kOut | kMass, false>(J.g, bx, by, lds);
            }
            // the chunk's LDS is reused by the next claim of this wave
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

}  // namespace iga
