// serve_batch.hpp -- kernels of the serving loop's batched iterations.
//
// The server keeps every admitted request that it can batch (a Petrov-Galerkin right-hand
// side or a lumped explicit step, support spans, every axis of at least 3p+1 elements) as
// a job and advances all of them together: one iteration is one short sequence of
// launches in which each right-hand-side job runs once and each step job takes its next
// step (continuous batching at the granularity of a step).  A job needs no context.  Its
// band rows are the element-unit rows of (p, nq) scaled by its element length: expanded
// into tables of its own when it is admitted (2D, 3D) or formed on the fly (1D).  The
// step's scale and source rows are expanded the same way.  Every value is formed by the
// expressions the per-axis tables are built from (tables.hpp), and the arithmetic of the
// rows is that of the single-problem kernels, so a batched job gives the bits of the same
// request run alone on a context.
#pragma once

#include "apply.hpp"
#include "apply3d.hpp"
#include "tables.hpp"

namespace iga {

constexpr int kServeBlock = 256;

// The unit whose range of blocks holds block b: blk0[] ascending (units own at least one
// block), blk0[0] = 0.  A 64-way search by the lanes of each wave, two rounds for up to
// 4096 units; every wave of the workgroup finds the same unit.
__device__ __forceinline__ int find_unit(const int* __restrict__ blk0, int n, int b)
{
    const int lane = (int)(threadIdx.x & 63);
    int lo = 0, cnt = n;   // the unit lies in [lo, lo + cnt)
    while (cnt > 1) {
        const int step = (cnt + 63) / 64;
        const int idx = lo + lane * step;
        const bool ok = idx < lo + cnt && blk0[idx] <= b;
        const unsigned long long m = __ballot(ok);   // a prefix of the lanes, lane 0 always
        const int last = 63 - __clzll(m);
        const int nlo = lo + last * step;
        cnt = min(step, lo + cnt - nlo);
        lo = nlo;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Set-up of newly admitted jobs: one unit per axis whose tables are expanded (kServeBlock
// rows per workgroup), or one copy (kServeBlock values per workgroup).
struct ExpandUnit {
    const double* gen;   // element-unit PG rows of (p, nq)
    double* M;           // [R][W] mass-type rows, or null
    double* D;           // [R][W] second-derivative rows (with M)
    double* S;           // [R] scale 1/|S_r| of the lumped step, or null
    double* F;           // [R] separable sine-source rows, or null
    const double* src;   // a copy unit: n values src -> dst (the fields above unused)
    double* dst;
    long long n;
    double lo, hi;
    int p, nq, ne, R;
    int ones;            // F = 1 (a step without source)
    int pad;
};

__global__ __launch_bounds__(kServeBlock) void serve_expand_kernel(const ExpandUnit* __restrict__ units,
                                                                   const int* __restrict__ blk0, int n)
{
    __shared__ double sgw[kMaxNq], sgs[kMaxNq];
    const int b = (int)blockIdx.x;
    const int k = find_unit(blk0, n, b);
    const ExpandUnit U = units[k];
    const long long i = (long long)(b - blk0[k]) * kServeBlock + threadIdx.x;
    if (U.src) {
        if (i < U.n) U.dst[i] = U.src[i];
        return;
    }
    const int p = U.p, W = 2 * p + 1;
    const double h = elem_len(U.lo, U.hi, U.ne), ih = elem_inv_len(U.lo, U.hi, U.ne);
    const bool sine = U.F && !U.ones;
    if (sine) {   // the Gauss rule of the axis, weights times the Jacobian
        const double* gq = U.gen + 2 * (size_t)(4 * p + 1) * W;   // w[nq] | s[nq]
        for (int q = (int)threadIdx.x; q < U.nq; q += kServeBlock) {
            sgw[q] = 0.5 * gq[q] * h;
            sgs[q] = gq[U.nq + q];
        }
        __syncthreads();
    }
    if (i >= U.R) return;
    const int r = (int)i;
    int s, l;
    support_span(r, p, U.ne, &s, &l);
    if (U.M) {
        double m[2 * kMaxP + 1], d[2 * kMaxP + 1];
        pg_generic_row(U.gen, p, r, U.R, h, ih, m, d);
        for (int t = 0; t < W; ++t) {
            U.M[(size_t)r * W + t] = m[t];
            U.D[(size_t)r * W + t] = d[t];
        }
    }
    if (U.S) U.S[r] = span_scale(s, l, U.ne, U.lo, U.hi);
    if (U.F) {
        double fs = 1.0;
        if (sine) {
            fs = 0.0;
            for (int e = s; e <= l; ++e) fs += elem_sine_sum(U.lo, U.hi, U.ne, e, U.nq, sgw, sgs);
        }
        U.F[r] = fs;
    }
}

// 1D jobs: one thread per row, the taps formed from the element-unit rows.
struct Job1D {
    const double* gen;   // element-unit PG rows of (p, p+1)
    const double* u;     // [N]
    double* out;         // RHS: Laplacian rows; step: the next iterate
    double* omass;       // RHS: mass rows; step: null
    const double* F;     // step: source rows, or null (no source)
    double lo, hi;
    double alpha, beta, gsep;
    int p, ne, step, pad;
};

template <int P>
__device__ __forceinline__ void serve1d_row(const Job1D& J, int r)
{
    constexpr int W = 2 * P + 1;
    const int N = J.ne + P;
    double mt[2 * kMaxP + 1], dt[2 * kMaxP + 1];
    pg_generic_row(J.gen, P, r, N, elem_len(J.lo, J.hi, J.ne), elem_inv_len(J.lo, J.hi, J.ne), mt, dt);
    double m = 0.0, d = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int j = r + k - P;
        const double uj = (j >= 0 && j < N) ? J.u[j] : 0.0;
        m = fma(mt[k], uj, m);
        d = fma(dt[k], uj, d);
    }
    ApplyArgs g = {};
    g.out = J.out;
    g.omass = J.omass;
    g.alpha = J.alpha;
    g.beta = J.beta;
    g.gsep = J.gsep;
    if (J.step) {
        int s, l;
        support_span(r, P, J.ne, &s, &l);
        finish_row<kOut | kScaleSrc>(g, r, m, d, span_scale(s, l, J.ne, J.lo, J.hi), J.F ? J.F[r] : 1.0);
    } else {
        finish_row<kOut | kMass>(g, r, m, d, 1.0, 1.0);
    }
}

__global__ __launch_bounds__(kServeBlock) void serve1d_kernel(const Job1D* __restrict__ jobs,
                                                              const int* __restrict__ blk0, int n)
{
    const int b = (int)blockIdx.x;
    const int k = find_unit(blk0, n, b);
    const Job1D J = jobs[k];
    const int r = (b - blk0[k]) * kServeBlock + (int)threadIdx.x;
    if (r >= J.ne + J.p) return;
    if (J.p == 2)
        serve1d_row<2>(J, r);
    else
        serve1d_row<3>(J, r);
}

// 3D jobs of one degree and output mode: the tiles of every job's plan, one workgroup
// each, the jobs' blocks numbered consecutively.
struct Job3D {
    ApplyArgs g;
    Plan3D pl;
};

template <int P, int MODE>
__global__ __launch_bounds__(kMaxNT3, 4) void serve3d_kernel(const Job3D* __restrict__ jobs,
                                                             const int* __restrict__ blk0, int n)
{
    const int b = (int)blockIdx.x;
    const int k = find_unit(blk0, n, b);
    const Job3D J = jobs[k];
    apply3d_tile<P, MODE>(J.g, J.pl, b - blk0[k]);
}

}  // namespace iga
