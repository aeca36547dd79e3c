// source.hpp -- right-hand sides of a source given at the Gauss points (a table with
// one value per Gauss point), Section 4.1: the paper's generation loops for the
// L2-projection right-hand side.
//
//   Petrov-Galerkin:  F_r = sum_{e in S_r} sum_q W_q f_q        (test = 1, never evaluated)
//   Galerkin:         F_i = sum_e sum_q W_q B_i(x_q) f_q         (test B_i at every point)
//
// Both run in two steps: a per-element reduction over the element's Gauss points
// (PG: one number; Galerkin: one number per local test function), then a gather of
// the element results into rows (PG: span sums one axis at a time).  Every gather reads
// the element results a row needs, so no atomics are used and the result does not
// depend on timing.
#pragma once

#include "common.hpp"

namespace iga {

struct SrcAxis {
    int ne, nq, np1, p;       // elements, Gauss points per element, local functions, degree
    int R;                    // rows of this axis
    const double* gw;         // [nq] weight * Jacobian (the same on every element)
    const double* cls;        // basis values by element class (see class_of)
    const int* first;         // [R] PG spans
    const int* last;
};

// W B_{e+a} at Gauss point q of element e
__device__ __forceinline__ double wbasis(const SrcAxis& A, int e, int q, int a)
{
    return A.gw[q] * A.cls[(((size_t)class_of(e, A.p, A.ne) * A.nq + q) * 3) * A.np1 + a];
}

struct SrcArgs {
    SrcAxis ax[3];            // axes beyond dim: ne = nq = np1 = R = 1, unit tables
    const double* table;      // (ne_z nq_z, ne_y nq_y, ne_x nq_x)
    double* elem;             // PG: [n_el] (then span sums); Galerkin: [np1^d][n_el]
    double* rows;             // (R_z, R_y, R_x)
};

__device__ __forceinline__ void elem_index(const SrcArgs& s, size_t idx, int e[3])
{
    e[0] = (int)(idx % s.ax[0].ne);
    e[1] = (int)((idx / s.ax[0].ne) % s.ax[1].ne);
    e[2] = (int)(idx / ((size_t)s.ax[0].ne * s.ax[1].ne));
}

// PG step 1: E_e = sum_q W_q f_q over the element's Gauss points.
__global__ void pg_src_elem_kernel(SrcArgs s, size_t nel)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nel) return;
    int e[3];
    elem_index(s, idx, e);
    const SrcAxis &X = s.ax[0], &Y = s.ax[1], &Z = s.ax[2];
    const size_t gx0 = (size_t)e[0] * X.nq, gy0 = (size_t)e[1] * Y.nq, gz0 = (size_t)e[2] * Z.nq;
    const size_t ngx = (size_t)X.ne * X.nq, ngy = (size_t)Y.ne * Y.nq;
    double acc = 0.0;
    for (int qz = 0; qz < Z.nq; ++qz)
        for (int qy = 0; qy < Y.nq; ++qy) {
            const double wyz = Z.gw[qz] * Y.gw[qy];
            const double* row = s.table + ((gz0 + qz) * ngy + gy0 + qy) * ngx + gx0;
            double t = 0.0;
            for (int qx = 0; qx < X.nq; ++qx) t = fma(X.gw[qx], row[qx], t);
            acc = fma(wyz, t, acc);
        }
    s.elem[idx] = acc;
}

// PG step 1 for NQ Gauss points along x (the common rules): the same sums in the same
// order, with the table read by 16-byte accesses.  A thread takes E consecutive elements
// of an x-line, E = 2 for odd NQ so that its share of a table row is a whole number of
// 16-byte pairs; consecutive threads read consecutive pairs of every row (a wave reads
// contiguous memory).  nunits: threads = ceil(ne_x / E) * ne_y * ne_z.
typedef double src_pair __attribute__((ext_vector_type(2), aligned(8)));

template <int NQ>
__global__ __launch_bounds__(kBlock) void pg_src_elem_vec_kernel(SrcArgs s, size_t nunits)
{
    constexpr int E = (NQ & 1) ? 2 : 1;
    constexpr int V = E * NQ / 2;   // pairs per table row
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nunits) return;
    const SrcAxis &X = s.ax[0], &Y = s.ax[1], &Z = s.ax[2];
    const int nux = (X.ne + E - 1) / E;
    const int ex0 = (int)(idx % (size_t)nux) * E;
    const size_t t = idx / (size_t)nux;
    const int ey = (int)(t % (size_t)Y.ne), ez = (int)(t / (size_t)Y.ne);
    const bool full = ex0 + E <= X.ne;   // else only element ex0 (the last of its line)
    double w[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) w[q] = X.gw[q];
    const size_t ngx = (size_t)X.ne * NQ, ngy = (size_t)Y.ne * Y.nq;
    const size_t gy0 = (size_t)ey * Y.nq, gz0 = (size_t)ez * Z.nq;
    double acc[E];
#pragma unroll
    for (int j = 0; j < E; ++j) acc[j] = 0.0;
    auto plane_row = [&](int qz, int qy) {
        const double wyz = Z.gw[qz] * Y.gw[qy];
        const double* row = s.table + ((gz0 + qz) * ngy + gy0 + qy) * ngx + (size_t)ex0 * NQ;
        double v[E * NQ];
        if (full) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const src_pair pr = *reinterpret_cast<const src_pair*>(row + 2 * k);
                v[2 * k] = pr.x;
                v[2 * k + 1] = pr.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < E * NQ; ++k) v[k] = k < NQ ? row[k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < E; ++j) {
            double tt = 0.0;
#pragma unroll
            for (int qx = 0; qx < NQ; ++qx) tt = fma(w[qx], v[j * NQ + qx], tt);
            acc[j] = fma(wyz, tt, acc[j]);
        }
    };
    // the rows in (qz, qy) order; with the rule of x on y (and z) the loops have
    // compile-time bounds, so the loads of a whole element are issued together
    if (Y.nq == NQ && Z.nq == NQ) {
#pragma unroll
        for (int qz = 0; qz < NQ; ++qz)
#pragma unroll
            for (int qy = 0; qy < NQ; ++qy) plane_row(qz, qy);
    } else if (Y.nq == NQ && Z.nq == 1) {
#pragma unroll
        for (int qy = 0; qy < NQ; ++qy) plane_row(0, qy);
    } else {
        for (int qz = 0; qz < Z.nq; ++qz)
#pragma unroll 4
            for (int qy = 0; qy < Y.nq; ++qy) plane_row(qz, qy);
    }
    const size_t e0 = ((size_t)ez * Y.ne + ey) * X.ne + ex0;
    s.elem[e0] = acc[0];
    if (E == 2 && full) s.elem[e0 + 1] = acc[E - 1];
}

// PG steps 1 and 2 along x in one pass, for support spans (every span inside
// [r - P, r]): the lanes of a wave hold the element sums of 128 consecutive elements of an
// x-line (two per lane, the same sums in the same order as pg_src_elem_vec_kernel) and
// form the span sums of the 128 - P rows whose spans lie among them from their own and
// their right neighbours' values (cross-lane shuffles, each sum in ascending element
// order, as src_span_sum_kernel forms it); consecutive waves of a line overlap by P
// elements.  out[line][rx] with line = ez ne_y + ey: the x-pass sums, or F_r in 1D.
// wpl: waves per x-line, ceil(R_x / (128 - P)); nwaves: wpl times the lines.
template <int NQ, int P>
__global__ __launch_bounds__(kBlock) void pg_src_elem_x_kernel(SrcArgs s, double* __restrict__ out, int wpl,
                                                               size_t nwaves)
{
    constexpr int E = 2;                   // elements per lane
    constexpr int S = 64 * E - P;          // rows per wave
    constexpr int K = (P + E - 1) / E + 1; // lanes whose values a row may need (itself and K-1 more)
    const size_t gw = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (gw >= nwaves) return;   // whole waves
    const int lane = (int)(threadIdx.x & 63);
    const SrcAxis &X = s.ax[0], &Y = s.ax[1], &Z = s.ax[2];
    const int w = (int)(gw % (size_t)wpl);
    const size_t line = gw / (size_t)wpl;
    const int ey = (int)(line % (size_t)Y.ne), ez = (int)(line / (size_t)Y.ne);
    const int e0 = w * S - P + lane * E;   // this lane's first element
    double wx[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) wx[q] = X.gw[q];
    const size_t ngx = (size_t)X.ne * NQ, ngy = (size_t)Y.ne * Y.nq;
    const size_t gy0 = (size_t)ey * Y.nq, gz0 = (size_t)ez * Z.nq;
    const bool full = e0 >= 0 && e0 + E <= X.ne;
    bool ok[E];
#pragma unroll
    for (int j = 0; j < E; ++j) ok[j] = e0 + j >= 0 && e0 + j < X.ne;
    double acc[E];
#pragma unroll
    for (int j = 0; j < E; ++j) acc[j] = 0.0;
    auto plane_row = [&](int qz, int qy) {
        const double wyz = Z.gw[qz] * Y.gw[qy];
        const double* row = s.table + ((gz0 + qz) * ngy + gy0 + qy) * ngx;
        double v[E * NQ];
        if (full) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const src_pair pr = *reinterpret_cast<const src_pair*>(row + (size_t)e0 * NQ + 2 * k);
                v[2 * k] = pr.x;
                v[2 * k + 1] = pr.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < E; ++j)
#pragma unroll
                for (int k = 0; k < NQ; ++k) v[j * NQ + k] = ok[j] ? row[(size_t)(e0 + j) * NQ + k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < E; ++j) {
            double tt = 0.0;
#pragma unroll
            for (int qx = 0; qx < NQ; ++qx) tt = fma(wx[qx], v[j * NQ + qx], tt);
            acc[j] = fma(wyz, tt, acc[j]);
        }
    };
    if (ok[0] || ok[E - 1]) {   // the rows in (qz, qy) order, compile-time bounds where the rules allow
        if (Y.nq == NQ && Z.nq == NQ) {
#pragma unroll
            for (int qz = 0; qz < NQ; ++qz)
#pragma unroll
                for (int qy = 0; qy < NQ; ++qy) plane_row(qz, qy);
        } else if (Y.nq == NQ && Z.nq == 1) {
#pragma unroll
            for (int qy = 0; qy < NQ; ++qy) plane_row(0, qy);
        } else {
            for (int qz = 0; qz < Z.nq; ++qz)
#pragma unroll 4
                for (int qy = 0; qy < Y.nq; ++qy) plane_row(qz, qy);
        }
    }
    // the values of this lane and the next K-1: element e0 + o at nb[o]
    double nb[K * E];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int j = 0; j < E; ++j) nb[k * E + j] = k == 0 ? acc[j] : __shfl_down(acc[j], (unsigned)k);
    double* const orow = out + line * (size_t)X.R;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int rx = w * S + lane * E + j;   // its span lies in elements e0 + j .. e0 + j + P
        if (lane * E + j >= S || rx >= X.R) continue;
        const int f = X.first[rx], l = X.last[rx];
        double sum = 0.0;
#pragma unroll
        for (int o = j; o <= j + P; ++o)
            if (e0 + o >= f && e0 + o <= l) sum += nb[o];
        orow[rx] = sum;
    }
}

// PG step 2, one axis at a time (the tensor span is a product of per-axis spans):
//   out[o][r][i] = sum_{e = first[r]}^{last[r]} in[o][e][i]
// for o < nouter, r < nout, i < ninner, in holding nin entries along the axis.  Applied
// along x, then y, then z: F_r = sum_{ez in Sz} sum_{ey in Sy} sum_{ex in Sx} E_e, each
// sum in ascending element order.  One thread per output; total = nouter nout ninner.
// I: the index type, 32-bit whenever the arrays allow (its divisions are far cheaper).
// Blocks are numbered XCD-aware: the outputs of neighbouring blocks share most of their
// inputs, which then come from one L2.
template <typename I>
__global__ __launch_bounds__(kBlock) void src_span_sum_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                              const int* __restrict__ first,
                                                              const int* __restrict__ last, int nin, int nout,
                                                              I ninner, I total)
{
    const I blk = (I)xcd_logical_block((int)blockIdx.x, (int)gridDim.x);
    const I idx = blk * (I)blockDim.x + (I)threadIdx.x;
    if (idx >= total) return;
    const I i = idx % ninner, t = idx / ninner;
    const I r = t % (I)nout, o = t / (I)nout;
    const double* src = in + ((size_t)o * (size_t)nin * (size_t)ninner + i);
    const int f = first[r], l = last[r];
    double acc = 0.0;
    for (int e0 = f; e0 <= l; e0 += 4) {   // four loads in flight, then the sums in order
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = e0 + k <= l ? src[(size_t)(e0 + k) * ninner] : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (e0 + k <= l) acc += v[k];
    }
    out[idx] = acc;
}

// Galerkin step 1: E_{e,a} = sum_q W_q B_{e+a}(x_q) f_q for the np1^dim local tests a,
// by sum factorization over the element's Gauss points:
//   tx[ax]          = sum_qx  W_x B_{ax}(x_qx) f_(qz,qy,qx)
//   sy[ay][ax]      = sum_qy  W_y B_{ay}(y_qy) tx[ax]
//   E[az][ay][ax]   = sum_qz  W_z B_{az}(z_qz) sy[ay][ax]
// (nq^d (p+1) + nq^(d-1) (p+1)^2 + ... products instead of nq^d (p+1)^d; the table is read
// once per element).  P: the degree of the mesh; axes beyond dim have one local function.
// NQ > 0: x and y both have NQ Gauss points, and the NQ x NQ table values of a z-plane of
// the element are loaded together before they are used (one wait per plane); NQ = 0:
// any rule, loops bounded at run time.
// The products W_q B_{e+a}(x_q) of every element class of the three axes are staged in
// LDS once per workgroup ([axis][class][q][a]); a thread reads those of its element's
// classes.
template <int P, int NQ>
__global__ __launch_bounds__(kBlock) void gal_src_elem_kernel(SrcArgs s, size_t nel)
{
    constexpr int Q = P + 1;
    constexpr int kAxisW = (2 * kMaxP + 1) * kMaxNq * (kMaxP + 1);
    __shared__ double wt[3 * kAxisW];
    for (int a = 0; a < 3; ++a) {
        const SrcAxis& A = s.ax[a];
        const int n = n_classes(A.p, A.ne) * A.nq * A.np1;
        for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) {
            const int j = i % A.np1, q = (i / A.np1) % A.nq, c = i / (A.np1 * A.nq);
            wt[a * kAxisW + i] = A.gw[q] * A.cls[(((size_t)c * A.nq + q) * 3) * A.np1 + j];
        }
    }
    __syncthreads();
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nel) return;
    int e[3];
    elem_index(s, idx, e);
    const SrcAxis &X = s.ax[0], &Y = s.ax[1], &Z = s.ax[2];
    const int nx = X.np1, ny = Y.np1, nz = Z.np1;   // Q or 1
    // this element's rows of the staged products: [q][a]
    const double* const wx = wt + (size_t)class_of(e[0], X.p, X.ne) * X.nq * nx;
    const double* const wy = wt + kAxisW + (size_t)class_of(e[1], Y.p, Y.ne) * Y.nq * ny;
    const double* const wz = wt + 2 * kAxisW + (size_t)class_of(e[2], Z.p, Z.ne) * Z.nq * nz;
    const size_t gx0 = (size_t)e[0] * X.nq, gy0 = (size_t)e[1] * Y.nq, gz0 = (size_t)e[2] * Z.nq;
    const size_t ngx = (size_t)X.ne * X.nq, ngy = (size_t)Y.ne * Y.nq;
    double acc[Q][Q][Q];
#pragma unroll
    for (int az = 0; az < Q; ++az)
#pragma unroll
        for (int ay = 0; ay < Q; ++ay)
#pragma unroll
            for (int ax = 0; ax < Q; ++ax) acc[az][ay][ax] = 0.0;
    for (int qz = 0; qz < Z.nq; ++qz) {
        double sy[Q][Q];
#pragma unroll
        for (int ay = 0; ay < Q; ++ay)
#pragma unroll
            for (int ax = 0; ax < Q; ++ax) sy[ay][ax] = 0.0;
        constexpr int NF = NQ > 0 ? NQ * NQ : 1;
        double fp[NF];   // NQ > 0: the plane's table values
        if constexpr (NQ > 0) {
#pragma unroll
            for (int qy = 0; qy < NQ; ++qy)
#pragma unroll
                for (int qx = 0; qx < NQ; ++qx)
                    fp[qy * NQ + qx] = s.table[((gz0 + qz) * ngy + gy0 + qy) * ngx + gx0 + qx];
        }
#pragma unroll
        for (int qy = 0; qy < (NQ > 0 ? NQ : Y.nq); ++qy) {
            const double* row = s.table + ((gz0 + qz) * ngy + gy0 + qy) * ngx + gx0;
            double tx[Q];
#pragma unroll
            for (int ax = 0; ax < Q; ++ax) tx[ax] = 0.0;
#pragma unroll
            for (int qx = 0; qx < (NQ > 0 ? NQ : X.nq); ++qx) {
                double f;
                if constexpr (NQ > 0)
                    f = fp[qy * NQ + qx];
                else
                    f = row[qx];
#pragma unroll
                for (int ax = 0; ax < Q; ++ax)
                    if (ax < nx) tx[ax] = fma(wx[qx * nx + ax], f, tx[ax]);
            }
#pragma unroll
            for (int ay = 0; ay < Q; ++ay) {
                if (ay >= ny) break;
                const double ty = wy[qy * ny + ay];
#pragma unroll
                for (int ax = 0; ax < Q; ++ax) sy[ay][ax] = fma(ty, tx[ax], sy[ay][ax]);
            }
        }
#pragma unroll
        for (int az = 0; az < Q; ++az) {
            if (az >= nz) break;
            const double tz = wz[qz * nz + az];
#pragma unroll
            for (int ay = 0; ay < Q; ++ay)
#pragma unroll
                for (int ax = 0; ax < Q; ++ax) acc[az][ay][ax] = fma(tz, sy[ay][ax], acc[az][ay][ax]);
        }
    }
    // one array per local test (element fastest): neighbouring threads store, and the
    // gather reads, neighbouring addresses
#pragma unroll
    for (int az = 0; az < Q; ++az)
#pragma unroll
        for (int ay = 0; ay < Q; ++ay)
#pragma unroll
            for (int ax = 0; ax < Q; ++ax)
                if (az < nz && ay < ny && ax < nx) s.elem[(size_t)((az * ny + ay) * nx + ax) * nel + idx] = acc[az][ay][ax];
}

// Galerkin rows by contracting the Gauss grid one axis at a time (x, then y, then z):
//   out[o][i][k] = sum_{a=0}^{P} [e = i - a in [0, ne)] sum_{q<NQ} W_q B_{e,a}(x_q) in[o][e NQ + q][k]
// where B_{e,a} is local function a of element e, so B_{e,a} = B_i; after the three axes
// out = F_i = sum_e sum_q W_q B_i(x_q) f_q.  Each Gauss value is read once (no per-element
// array of (p+1)^d values), and the weighted basis values of the axis' element classes
// are staged in LDS per workgroup.  Used when every axis has 2 to 4 Gauss points.
template <int P, int NQ>
__device__ __forceinline__ const double* gal_stage_axis(const SrcAxis& A, double* wt)
{
    constexpr int Q = P + 1;
    const int n = n_classes(A.p, A.ne) * NQ * Q;
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) {
        const int a = i % Q, q = (i / Q) % NQ, c = i / (Q * NQ);
        wt[i] = A.gw[q] * A.cls[(((size_t)c * NQ + q) * 3) * Q + a];
    }
    __syncthreads();
    return wt;
}

// The x contraction, straight from the table: a lane forms the P+1 local sums of one
// element (t[a] = sum_q W_q B_{e,a} f_q, its NQ values read once) and row i takes
// t_{i-a}[a] from the lane a places to its left (cross-lane shuffles); the waves of a
// Gauss-point row (line = gz ngy + gy) overlap by P elements.  out[line][i], i < N_x.
template <int P, int NQ>
__global__ __launch_bounds__(kBlock) void gal_src_x_kernel(SrcArgs s, double* __restrict__ out, int wpl,
                                                           size_t nwaves)
{
    constexpr int Q = P + 1, S = 64 - P;
    __shared__ double wt[(2 * kMaxP + 1) * kMaxNq * (kMaxP + 1)];
    const SrcAxis& X = s.ax[0];
    const double* const w = gal_stage_axis<P, NQ>(X, wt);
    const size_t gw = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (gw >= nwaves) return;   // whole waves
    const int lane = (int)(threadIdx.x & 63);
    const int wv = (int)(gw % (size_t)wpl);
    const size_t line = gw / (size_t)wpl;
    const int e = wv * S - P + lane;
    const bool ok = e >= 0 && e < X.ne;
    double t[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) t[a] = 0.0;
    if (ok) {
        const double* row = s.table + line * (size_t)X.ne * NQ + (size_t)e * NQ;
        double f[NQ];
        if constexpr ((NQ & 1) == 0) {
#pragma unroll
            for (int k = 0; k < NQ / 2; ++k) {
                const src_pair pr = *reinterpret_cast<const src_pair*>(row + 2 * k);
                f[2 * k] = pr.x;
                f[2 * k + 1] = pr.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q) f[q] = row[q];
        }
        const double* wc = w + (size_t)class_of(e, X.p, X.ne) * NQ * Q;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int a = 0; a < Q; ++a) t[a] = fma(wc[q * Q + a], f[q], t[a]);
    }
    double nb[Q];   // nb[a] = t[a] of the lane a places to the left (element e - a)
#pragma unroll
    for (int a = 0; a < Q; ++a) nb[a] = a == 0 ? t[0] : __shfl_up(t[a], (unsigned)a);
    const int i = e;   // the row of this lane: lanes P .. 63 hold rows wv S .. wv S + S - 1
    if (lane < P || i >= X.R) return;
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a)
        if (i - a >= 0 && i - a < X.ne) sum += nb[a];
    out[line * (size_t)X.R + i] = sum;
}

// The y or z contraction of an array (outer, ne NQ, ninner) into (outer, N, ninner): one
// thread per output, all (P+1) NQ loads issued before the sums (in the order a, q).
template <int P, int NQ, typename I>
__global__ __launch_bounds__(kBlock) void gal_src_axis_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                              SrcAxis A, I ninner, I total)
{
    constexpr int Q = P + 1;
    __shared__ double wt[(2 * kMaxP + 1) * kMaxNq * (kMaxP + 1)];
    const double* const w = gal_stage_axis<P, NQ>(A, wt);
    // XCD-aware block numbering: neighbouring rows read overlapping Gauss rows from one L2
    const I blk = (I)xcd_logical_block((int)blockIdx.x, (int)gridDim.x);
    const I idx = blk * (I)blockDim.x + (I)threadIdx.x;
    if (idx >= total) return;
    const I k = idx % ninner, t = idx / ninner;
    const I i = t % (I)A.R, o = t / (I)A.R;
    const double* src = in + ((size_t)o * A.ne * NQ) * (size_t)ninner + k;
    double v[Q][NQ];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int e = (int)i - a;
        const bool ok = e >= 0 && e < A.ne;
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[a][q] = ok ? src[((size_t)e * NQ + q) * ninner] : 0.0;
    }
    double sum = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int e = (int)i - a;
        if (e < 0 || e >= A.ne) continue;
        const double* wc = w + (size_t)class_of(e, A.p, A.ne) * NQ * Q;
        double ta = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) ta = fma(wc[q * Q + a], v[a][q], ta);
        sum += ta;
    }
    out[idx] = sum;
}

// Galerkin step 2: F_i = sum over the elements e = i - a (a local index per axis), the
// terms in the order (az, ay, ax); all loads of a row are issued before the sums.
// P: the degree of the mesh (axes beyond dim have one local function).
template <int P>
__global__ __launch_bounds__(kBlock) void gal_src_rows_kernel(SrcArgs s, size_t nrows)
{
    constexpr int Q = P + 1;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows) return;
    const SrcAxis &X = s.ax[0], &Y = s.ax[1], &Z = s.ax[2];
    const int ix = (int)(idx % X.R);
    const int iy = (int)((idx / X.R) % Y.R);
    const int iz = (int)(idx / ((size_t)X.R * Y.R));
    const size_t nel = (size_t)X.ne * Y.ne * Z.ne;
    double v[Q][Q][Q];
#pragma unroll
    for (int az = 0; az < Q; ++az)
#pragma unroll
        for (int ay = 0; ay < Q; ++ay)
#pragma unroll
            for (int ax = 0; ax < Q; ++ax) {
                const int ez = iz - az, ey = iy - ay, ex = ix - ax;
                const bool ok = az < Z.np1 && ay < Y.np1 && ax < X.np1 && ez >= 0 && ez < Z.ne && ey >= 0 &&
                                ey < Y.ne && ex >= 0 && ex < X.ne;
                v[az][ay][ax] = ok ? s.elem[(size_t)((az * Y.np1 + ay) * X.np1 + ax) * nel +
                                            ((size_t)ez * Y.ne + ey) * X.ne + ex]
                                   : 0.0;
            }
    double acc = 0.0;
#pragma unroll
    for (int az = 0; az < Q; ++az)
#pragma unroll
        for (int ay = 0; ay < Q; ++ay)
#pragma unroll
            for (int ax = 0; ax < Q; ++ax) {
                const int ez = iz - az, ey = iy - ay, ex = ix - ax;
                if (az < Z.np1 && ay < Y.np1 && ax < X.np1 && ez >= 0 && ez < Z.ne && ey >= 0 && ey < Y.ne &&
                    ex >= 0 && ex < X.ne)
                    acc += v[az][ay][ax];
            }
    s.rows[idx] = acc;
}

}  // namespace iga
