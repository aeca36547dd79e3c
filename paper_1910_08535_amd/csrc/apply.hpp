// apply.hpp -- the hot kernels: generation of Galerkin / Petrov-Galerkin rows
//   out_r = S(r) ( alpha int T_r u_h + beta int T_r Lap u_h + source )
// for tensor-product B-splines, evaluated by sum factorization.
//
// The Gauss sums of every row are re-associated into banded 1D factors (built once by
// tables.hpp from the basis values at the Gauss points): on each axis, row r of the
// mass-type factor is sum_q W T_r B_j and of the operator factor sum_q W T_r B_j''
// (T_r = 1 on the span S_r for the Petrov-Galerkin form, Section 2 -- the test
// function is never evaluated).  The d-dimensional rows are then Kronecker products
// (Section 3), applied axis by axis:
//   x pass: A = Mx u, B = Dx u
//   y pass: C = My A, E = Dy A + My B
//   z pass: mass = Mz C, lap = Dz C + Mz E
// This is an exact re-association of the same finite sums, so it agrees with the
// Gauss-point-wise evaluation up to round-off.  Every pass is a (2p+1)-tap stencil
// whose taps vary only in the first and last p rows of an axis (open knots).
//
// Memory: u is read once from HBM per tile plus p-wide halos (served by L2), rows are
// written once.  The kernels are HBM-bound for p = 2 and near the FP64 ridge for
// p = 3 in 3D; the per-tile data stays in LDS (x pass) and registers (z ring).
#pragma once

#include "common.hpp"

namespace iga {

__device__ __forceinline__ void finish_row(const ApplyArgs& g, size_t idx, double mass, double lap,
                                           double scale, double fsep)
{
    if (g.omass) g.omass[idx] = mass;
    if (g.out) {
        double v = g.alpha * mass + g.beta * lap;
        if (g.gsep != 0.0) v += g.gsep * fsep;
        if (g.farr) v += g.garr * g.farr[idx];
        g.out[idx] = scale * v;
    }
}

__device__ __forceinline__ double axis_scale(const AxisOp& a, int r)
{
    return a.S ? a.S[r] : 1.0;
}

__device__ __forceinline__ double axis_src(const AxisOp& a, int r)
{
    return a.F ? a.F[r] : 1.0;
}

// ---------------------------------------------------------------------------------
// 1D: one thread per row, coefficients through the L1/L2 caches.
// ---------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void apply1d_kernel(ApplyArgs g)
{
    constexpr int W = 2 * P + 1;
    const AxisOp X = g.ax[0];
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= X.R) return;
    double m = 0.0, d = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int j = r + k - P;
        const double uj = (j >= 0 && j < X.N) ? g.u[j] : 0.0;
        m = fma(X.M[(size_t)r * W + k], uj, m);
        d = fma(X.D[(size_t)r * W + k], uj, d);
    }
    finish_row(g, r, m, d, axis_scale(X, r), axis_src(X, r));
}

// ---------------------------------------------------------------------------------
// Shared pieces of the 2D / 3D tiles: a plane tile of (TY+2P) x (TX+2P) coefficients
// in LDS, the x pass into LDS, and the y pass of one output row.
// ---------------------------------------------------------------------------------
template <int P, int TX, int TY>
struct PlaneTile {
    static constexpr int W = 2 * P + 1;
    static constexpr int HX = TX + 2 * P;
    static constexpr int HY = TY + 2 * P;
};

// Loads the coefficient plane rows y0-P .. y0+TY+P-1, columns x0-P .. x0+TX+P-1 of
// `plane` (Ny x Nx, x fastest) into su; zero outside the array.
template <int P, int TX, int TY>
__device__ __forceinline__ void load_plane(double* __restrict__ su, const double* __restrict__ plane,
                                           int x0, int y0, int Nx, int Ny)
{
    using T = PlaneTile<P, TX, TY>;
    for (int i = threadIdx.x; i < T::HY * T::HX; i += kBlock) {
        const int iy = i / T::HX, ix = i - iy * T::HX;
        const int gy = y0 - P + iy, gx = x0 - P + ix;
        double v = 0.0;
        if (gy >= 0 && gy < Ny && gx >= 0 && gx < Nx) v = plane[(size_t)gy * Nx + gx];
        su[i] = v;
    }
}

// x pass over all HY rows of the tile: A = Mx u, B = Dx u for this lane's column.
template <int P, int TX, int TY>
__device__ __forceinline__ void x_pass(const double* __restrict__ su, double* __restrict__ sA,
                                       double* __restrict__ sB, const double (&mx)[2 * P + 1],
                                       const double (&dx)[2 * P + 1], int lane, int wave)
{
    using T = PlaneTile<P, TX, TY>;
    for (int iy = wave; iy < T::HY; iy += kBlock / 64) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int k = 0; k < T::W; ++k) {
            const double v = su[iy * T::HX + lane + k];
            a = fma(mx[k], v, a);
            b = fma(dx[k], v, b);
        }
        sA[iy * TX + lane] = a;
        sB[iy * TX + lane] = b;
    }
}

// ---------------------------------------------------------------------------------
// 2D: output tile of 64 x TY rows; one lane per output column.
// ---------------------------------------------------------------------------------
template <int P, int TY>
__global__ __launch_bounds__(kBlock) void apply2d_kernel(ApplyArgs g, TileGrid tg)
{
    constexpr int TX = 64;
    using T = PlaneTile<P, TX, TY>;
    constexpr int W = T::W;
    __shared__ double su[T::HY * T::HX];
    __shared__ double sA[T::HY * TX];
    __shared__ double sB[T::HY * TX];

    const AxisOp X = g.ax[0], Y = g.ax[1];
    const int L = xcd_logical_block(blockIdx.x, tg.nblk);
    const int bx = L % tg.tx, by = L / tg.tx;
    const int x0 = bx * TX, y0 = by * TY;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    load_plane<P, TX, TY>(su, g.u, x0, y0, X.N, Y.N);

    const int gx = x0 + lane;
    const bool colok = gx < X.R;
    double mx[W], dx[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        mx[k] = colok ? X.M[(size_t)gx * W + k] : 0.0;
        dx[k] = colok ? X.D[(size_t)gx * W + k] : 0.0;
    }
    const double sx = colok ? axis_scale(X, gx) : 0.0;
    const double fx = colok ? axis_src(X, gx) : 0.0;
    __syncthreads();
    x_pass<P, TX, TY>(su, sA, sB, mx, dx, lane, wave);
    __syncthreads();

    for (int oy = wave; oy < TY; oy += kBlock / 64) {
        const int gy = y0 + oy;
        if (gy >= Y.R) break;
        double mass = 0.0, lapy = 0.0, lapx = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const double my = Y.M[(size_t)gy * W + k];
            const double dy = Y.D[(size_t)gy * W + k];
            const double a = sA[(oy + k) * TX + lane];
            const double b = sB[(oy + k) * TX + lane];
            mass = fma(my, a, mass);
            lapy = fma(dy, a, lapy);
            lapx = fma(my, b, lapx);
        }
        if (colok)
            finish_row(g, (size_t)gy * X.R + gx, mass, lapx + lapy, sx * axis_scale(Y, gy),
                       fx * axis_src(Y, gy));
    }
}

// ---------------------------------------------------------------------------------
// 3D: in-plane output tile of 64 x 8, streamed along z over a chunk of TZ output
// planes.  Each input plane goes through the x pass (LDS) and the y pass; the y-pass
// results of the last 2P+1 planes stay in a register ring from which the z pass forms
// one output plane per input plane.
// ---------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void apply3d_kernel(ApplyArgs g, TileGrid tg)
{
    constexpr int TX = 64, TY = 8;
    using T = PlaneTile<P, TX, TY>;
    constexpr int W = T::W;
    constexpr int Q = TY / (kBlock / 64);   // output rows per wave
    __shared__ double su[T::HY * T::HX];
    __shared__ double sA[T::HY * TX];
    __shared__ double sB[T::HY * TX];

    const AxisOp X = g.ax[0], Y = g.ax[1], Z = g.ax[2];
    const int L = xcd_logical_block(blockIdx.x, tg.nblk);
    const int bx = L % tg.tx;
    const int by = (L / tg.tx) % tg.ty;
    const int bz = L / (tg.tx * tg.ty);
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * tg.TZ;
    const int z1 = min(z0 + tg.TZ, Z.R);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const size_t plane_in = (size_t)X.N * Y.N;

    const int gx = x0 + lane;
    const bool colok = gx < X.R;
    double mx[W], dx[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        mx[k] = colok ? X.M[(size_t)gx * W + k] : 0.0;
        dx[k] = colok ? X.D[(size_t)gx * W + k] : 0.0;
    }
    const double sx = colok ? axis_scale(X, gx) : 0.0;
    const double fx = colok ? axis_src(X, gx) : 0.0;

    double rc[W][Q], re[W][Q];
#pragma unroll
    for (int s = 0; s < W; ++s)
#pragma unroll
        for (int j = 0; j < Q; ++j) rc[s][j] = re[s][j] = 0.0;

    for (int zb = z0 - P; zb < z1 + P; zb += W) {
#pragma unroll
        for (int ph = 0; ph < W; ++ph) {
            const int zi = zb + ph;
            if (zi >= z1 + P) break;
            if (zi >= 0 && zi < Z.N) {
                // su was last read by the previous x pass, which every thread finished
                // before the barrier that preceded the previous y pass.
                load_plane<P, TX, TY>(su, g.u + (size_t)zi * plane_in, x0, y0, X.N, Y.N);
                __syncthreads();
                x_pass<P, TX, TY>(su, sA, sB, mx, dx, lane, wave);
                __syncthreads();
#pragma unroll
                for (int j = 0; j < Q; ++j) {
                    const int oy = wave + j * (kBlock / 64);
                    const int gy = min(y0 + oy, Y.R - 1);
                    double c = 0.0, e = 0.0;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const double my = Y.M[(size_t)gy * W + k];
                        const double dy = Y.D[(size_t)gy * W + k];
                        const double a = sA[(oy + k) * TX + lane];
                        const double b = sB[(oy + k) * TX + lane];
                        c = fma(my, a, c);
                        e = fma(dy, a, e);
                        e = fma(my, b, e);
                    }
                    rc[ph][j] = c;
                    re[ph][j] = e;
                }
            } else {
#pragma unroll
                for (int j = 0; j < Q; ++j) rc[ph][j] = re[ph][j] = 0.0;
            }
            const int zo = zi - P;
            if (zo >= z0) {
                const double sz = axis_scale(Z, zo), fz = axis_src(Z, zo);
#pragma unroll
                for (int j = 0; j < Q; ++j) {
                    double mass = 0.0, lap = 0.0;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const int s = (ph + 1 + k) % W;   // plane zo - P + k
                        const double mz = Z.M[(size_t)zo * W + k];
                        const double dz = Z.D[(size_t)zo * W + k];
                        mass = fma(mz, rc[s][j], mass);
                        lap = fma(dz, rc[s][j], lap);
                        lap = fma(mz, re[s][j], lap);
                    }
                    const int gy = y0 + wave + j * (kBlock / 64);
                    if (colok && gy < Y.R)
                        finish_row(g, ((size_t)zo * Y.R + gy) * X.R + gx, mass, lap,
                                   sx * axis_scale(Y, gy) * sz, fx * axis_src(Y, gy) * fz);
                }
            }
        }
    }
}

// Rows without a u-term: out_r = S(r) ( gsep prod_a F_a(r_a) + garr farr_r ).
__global__ void rows_only_kernel(ApplyArgs g, int dim, size_t nrows)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows) return;
    const int rx = (int)(idx % g.ax[0].R);
    const int ry = dim > 1 ? (int)((idx / g.ax[0].R) % g.ax[1].R) : 0;
    const int rz = dim > 2 ? (int)(idx / ((size_t)g.ax[0].R * g.ax[1].R)) : 0;
    double s = axis_scale(g.ax[0], rx), f = axis_src(g.ax[0], rx);
    if (dim > 1) { s *= axis_scale(g.ax[1], ry); f *= axis_src(g.ax[1], ry); }
    if (dim > 2) { s *= axis_scale(g.ax[2], rz); f *= axis_src(g.ax[2], rz); }
    finish_row(g, idx, 0.0, 0.0, s, f);
}

__global__ void copy_kernel(double* __restrict__ dst, const double* __restrict__ src, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace iga
