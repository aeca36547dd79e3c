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
// written once.  The 1D and 2D kernels live here; the 3D kernel (z pass first) is in
// apply3d.hpp.
#pragma once

#include "common.hpp"
#include "tables.hpp"

namespace iga {

// Output modes (template parameter of the kernels): which arrays a launch writes.
enum : int {
    kOut = 1,       // out_r = alpha mass + beta lap  [with the terms below]
    kMass = 2,      // omass_r = mass
    kFarr = 4,      // add garr * farr_r
    kScaleSrc = 8   // out_r = S(r) ( ... + gsep prod_a F_a(r_a) ): scaled rows / separable source
};

// S and F always point at real tables (a table of ones where the launch has none), so
// the only branches left are the compile-time output modes.
template <int MODE>
__device__ __forceinline__ void finish_row(const ApplyArgs& g, size_t idx, double mass, double lap,
                                           double scale, double fsep)
{
    if constexpr ((MODE & kMass) != 0) g.omass[idx] = mass;
    if constexpr ((MODE & kOut) != 0) {
        double v = fma(g.alpha, mass, g.beta * lap);
        if constexpr ((MODE & kScaleSrc) != 0) v = fma(g.gsep, fsep, v);
        if constexpr ((MODE & kFarr) != 0) v = fma(g.garr, g.farr[idx], v);
        if constexpr ((MODE & kScaleSrc) != 0) v *= scale;
        g.out[idx] = v;
    }
}

// The rows idx and idx + 1 (the second only when `two`) with one 16-byte access per array
// where both exist.
template <int MODE>
__device__ __forceinline__ double row_value(const ApplyArgs& g, double mass, double lap, double scale,
                                            double fsep, double farr)
{
    double v = fma(g.alpha, mass, g.beta * lap);
    if constexpr ((MODE & kScaleSrc) != 0) v = fma(g.gsep, fsep, v);
    if constexpr ((MODE & kFarr) != 0) v = fma(g.garr, farr, v);
    if constexpr ((MODE & kScaleSrc) != 0) v *= scale;
    return v;
}

template <int MODE>
__device__ __forceinline__ void finish_pair(const ApplyArgs& g, size_t idx, double m0, double l0, double s0,
                                            double f0, double m1, double l1, double s1, double f1, bool two)
{
    typedef double pair_t __attribute__((ext_vector_type(2), aligned(8)));
    if (two) {
        if constexpr ((MODE & kMass) != 0) *reinterpret_cast<pair_t*>(g.omass + idx) = pair_t{m0, m1};
        if constexpr ((MODE & kOut) != 0) {
            double a0 = 0.0, a1 = 0.0;
            if constexpr ((MODE & kFarr) != 0) {
                const pair_t fa = *reinterpret_cast<const pair_t*>(g.farr + idx);
                a0 = fa.x;
                a1 = fa.y;
            }
            *reinterpret_cast<pair_t*>(g.out + idx) =
                pair_t{row_value<MODE>(g, m0, l0, s0, f0, a0), row_value<MODE>(g, m1, l1, s1, f1, a1)};
        }
    } else {
        finish_row<MODE>(g, idx, m0, l0, s0, f0);
    }
}

// ---------------------------------------------------------------------------------
// 1D: one thread per row, coefficients through the L1/L2 caches.
// ---------------------------------------------------------------------------------
template <int P, int MODE>
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
    finish_row<MODE>(g, r, m, d, X.S[r], X.F[r]);
}

// 1D PG rows of support spans on an axis of at least 3p+1 elements: the taps are formed
// from the element-unit rows of (p, nq) (tables.hpp), the values the axis' own band
// tables hold, so the rows are those of apply1d_kernel bit for bit while each row reads
// 8 bytes of coefficients (and its scale and source factors) instead of 2(2p+1) taps.
template <int P, int MODE>
__global__ __launch_bounds__(kBlock) void apply1d_gen_kernel(ApplyArgs g, const double* gen, double h, double ih)
{
    constexpr int W = 2 * P + 1;
    const AxisOp X = g.ax[0];
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= X.R) return;
    double mt[2 * kMaxP + 1], dt[2 * kMaxP + 1];
    pg_generic_row(gen, P, r, X.R, h, ih, mt, dt);
    double m = 0.0, d = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int j = r + k - P;
        const double uj = (j >= 0 && j < X.N) ? g.u[j] : 0.0;
        m = fma(mt[k], uj, m);
        d = fma(dt[k], uj, d);
    }
    finish_row<MODE>(g, r, m, d, X.S[r], X.F[r]);
}

// ---------------------------------------------------------------------------------
// Buffer addressing.  A buffer resource carries the array's size; the hardware returns
// 0 for loads outside it and drops stores outside it, so edge tiles need no branches:
// an index outside the array is given the offset kOOB.
// ---------------------------------------------------------------------------------
typedef int iv2 __attribute__((ext_vector_type(2)));
constexpr unsigned kOOB = 0xffffffffu;

// Loads through the constant address space: with a wave-uniform address the compiler
// issues scalar loads.
typedef const __attribute__((address_space(4))) double* cdp;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void* p, size_t n_doubles)
{
    const size_t bytes = n_doubles * sizeof(double);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                             (int)(bytes > 0xffffffffull ? 0xffffffffull : bytes),
                                             0x00020000);
}

__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned byte_off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
}

// Cache policy of a buffer store: kStream marks it non-temporal, for outputs that
// this kernel never reads back (their lines then do not displace the halo rows of
// the input that neighbouring tiles still have to fetch).
constexpr int kKeep = 0;
constexpr int kStream = 2;

template <int POLICY = kKeep>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned byte_off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(iv2, v), r, (int)byte_off, 0, POLICY);
}

typedef int iv4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ dv2 bload2(__amdgpu_buffer_rsrc_t r, unsigned byte_off)
{
    return __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0));
}

template <int POLICY = kKeep>
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, unsigned byte_off, double a, double b)
{
    dv2 v;
    v.x = a;
    v.y = b;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(iv4, v), r, (int)byte_off, 0, POLICY);
}

// byte offset of element (row, col) of a rows x cols array, kOOB outside it
__device__ __forceinline__ unsigned boff(int row, int col, int rows, int cols)
{
    return (row >= 0 && row < rows && col >= 0 && col < cols)
               ? (unsigned)(((unsigned)row * (unsigned)cols + (unsigned)col) * 8u)
               : kOOB;
}

// ---------------------------------------------------------------------------------
// 2D: one wave per workgroup handles a strip of 128 output columns (two adjacent
// columns per lane) over a chunk of TY output rows.
//   1. all TY+2P input rows of the chunk are requested at once (128 values plus a halo
//      of P on each side per row; buffer bounds zero whatever lies outside u);
//   2. each row lands in an LDS row buffer as soon as its loads are in;
//   3. per row, the x pass (A = Mx u, B = Dx u) reads the lane's 2P+2 neighbours with
//      128-bit LDS reads; the last 2P+1 rows of (A, B) stay in a register ring and the
//      y pass (mass = My A, lap = Dy A + My B) forms one output row per input row.
// The row loop is unrolled at compile time (ring slots are registers, memory counters
// exact) and the code is branch-free: halo lanes, array edges and the band rows of
// the chunk are all handled by buffer bounds and spare LDS slots.
// ---------------------------------------------------------------------------------
// LDS doubles one 2D chunk needs
template <int P, int TY>
struct Chunk2D {
    static constexpr int W = 2 * P + 1;
    static constexpr int NR = TY + 2 * P;          // input rows of a chunk
    static constexpr int SW = 128;                 // strip width
    static constexpr int RBW = SW + 2 * P + 2;     // columns x0-P .. x0+SW+P-1, 2 spare slots
    static constexpr int CW = 2 * W + 2;           // band values per row: M[W], D[W], S, F
    static constexpr int NCV = (TY * CW + 63) / 64;
    static constexpr int LDS = NR * RBW + NCV * 64;
    static_assert(RBW % 2 == 0 && CW % 2 == 0, "16-byte LDS rows");
};

// One chunk: strip bx (output columns 128 bx ..) and rows TY by .. of one problem.
// lds: Chunk2D<P, TY>::LDS doubles, 16-byte aligned, private to the calling wave.
// DMA: even rows at even P load straight into LDS (below); the persistent batch kernel
// keeps the register path, which measured faster there.  YIN: every output row of the
// chunk is interior, so the y taps are one row for all of them, read with uniform loads
// (the chunk's band rows are then staged only when the step's S and F factors need them).
template <int P, int TY, int MODE, bool VEC, bool DMA = false, bool YIN = false>
__device__ __forceinline__ void apply2d_chunk(const ApplyArgs& g, int bx, int by, double* lds)
{
    using C = Chunk2D<P, TY>;
    constexpr int W = C::W, NR = C::NR, SW = C::SW, RBW = C::RBW, CW = C::CW, NCV = C::NCV;
    double (*rb)[RBW] = reinterpret_cast<double (*)[RBW]>(lds);
    double* cy = lds + NR * RBW;
    const AxisOp &X = g.ax[0], &Y = g.ax[1];
    const int x0 = bx * SW, y0 = by * TY;
    const int lane = threadIdx.x;
    const int Nx = X.N, Ny = Y.N;

    // x factors of the lane's two output columns
    const int c0 = x0 + 2 * lane;   // the lane's first column
    const int xr0 = c0, xr1 = c0 + 1;
    const auto rxm = buf(X.M, (size_t)X.R * W), rxd = buf(X.D, (size_t)X.R * W);
    double m0[W], d0[W], m1[W], d1[W];
    if (x0 >= X.ilo && x0 + SW - 1 <= X.ihi) {
        // every column of the strip is interior: one row for all lanes, read with uniform
        // (scalar) loads instead of 4W vector loads per lane
        const cdp um = (cdp)(X.M + (size_t)X.ilo * W), ud = (cdp)(X.D + (size_t)X.ilo * W);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            m0[k] = m1[k] = um[k];
            d0[k] = d1[k] = ud[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            m0[k] = bload(rxm, xr0 < X.R ? (unsigned)(xr0 * W + k) * 8u : kOOB);
            d0[k] = bload(rxd, xr0 < X.R ? (unsigned)(xr0 * W + k) * 8u : kOOB);
            m1[k] = bload(rxm, xr1 < X.R ? (unsigned)(xr1 * W + k) * 8u : kOOB);
            d1[k] = bload(rxd, xr1 < X.R ? (unsigned)(xr1 * W + k) * 8u : kOOB);
        }
    }
    double sx0 = 1.0, sx1 = 1.0, fx0 = 1.0, fx1 = 1.0;
    if constexpr ((MODE & kScaleSrc) != 0) {
        const auto rxs = buf(X.S, X.R), rxf = buf(X.F, X.R);
        sx0 = bload(rxs, xr0 < X.R ? (unsigned)xr0 * 8u : kOOB);
        sx1 = bload(rxs, xr1 < X.R ? (unsigned)xr1 * 8u : kOOB);
        fx0 = bload(rxf, xr0 < X.R ? (unsigned)xr0 * 8u : kOOB);
        fx1 = bload(rxf, xr1 < X.R ? (unsigned)xr1 * 8u : kOOB);
    }
    // band rows of the chunk: cy[j*CW + k]; every lane loads from each table with the
    // offset of the table that holds value k (the others read 0 out of bounds)
    // kDma (below): the band rows are stored after the input rows are issued, so that no
    // load waits for another
    constexpr bool kDma = DMA && VEC && (P % 2) == 0;
    constexpr bool kCy = !YIN || (MODE & kScaleSrc) != 0;   // the chunk's band rows are read
    double cv[NCV];
    if constexpr (kCy) {
        const auto rym = buf(Y.M, (size_t)Y.R * W), ryd = buf(Y.D, (size_t)Y.R * W);
        const auto rys = buf(Y.S, Y.R), ryf = buf(Y.F, Y.R);
#pragma unroll
        for (int c = 0; c < NCV; ++c) {
            const int i = lane + 64 * c;
            const int j = i / CW, k = i - j * CW;
            const int yr = y0 + j;
            const bool ok = i < TY * CW && yr < Y.R;
            const unsigned om = ok && k < W ? (unsigned)(yr * W + k) * 8u : kOOB;
            const unsigned od = ok && k >= W && k < 2 * W ? (unsigned)(yr * W + k - W) * 8u : kOOB;
            const unsigned os = ok && k == 2 * W ? (unsigned)yr * 8u : kOOB;
            const unsigned of = ok && k == 2 * W + 1 ? (unsigned)yr * 8u : kOOB;
            cv[c] = bload(rym, om) + bload(ryd, od) + bload(rys, os) + bload(ryf, of);
        }
        if constexpr (!kDma) {
#pragma unroll
            for (int c = 0; c < NCV; ++c) cy[lane + 64 * c] = cv[c];
        }
    }

    // 1. input rows (issued after the band loads: the memory counter retires in
    //    order, so the first FMA then waits for its factors, not for every row): the lane's two columns and one halo column (lanes < 2P)
    const auto ru = buf(g.u, (size_t)Nx * Ny);
    const int ch = lane < P ? x0 - P + lane : x0 + SW + lane - P;
    const bool ok0 = c0 < Nx, ok1 = c0 + 1 < Nx, okh = lane < 2 * P && ch >= 0 && ch < Nx;
    // kDma: rows of even length with an even halo width: each lane's pair goes from memory
    // straight into its 16-byte LDS slot (buffer load to LDS; lane l writes 16 bytes at the
    // row's slot P + 2l, out-of-range lanes write zeros), so the rows hold no registers
    typedef __attribute__((address_space(3))) void* lds_ptr;
    double v0[kDma ? 1 : NR], v1[kDma ? 1 : NR], vh[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int yi = y0 - P + i;
        const bool rowok = yi >= 0 && yi < Ny;
        const unsigned rowoff = (unsigned)yi * (unsigned)Nx;
        if constexpr (kDma) {
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ru, (lds_ptr)&rb[i][P], 16,
                                                     rowok && ok0 ? (rowoff + c0) * 8u : kOOB, 0, 0, 0);
        } else if constexpr (VEC) {   // rows of even length: the lane's pair is 16-byte aligned
            const dv2 v = bload2(ru, rowok && ok0 ? (rowoff + c0) * 8u : kOOB);
            v0[i] = v.x;
            v1[i] = v.y;
        } else {
            // rows of odd length: the pair is one 8-byte aligned 16-byte access; a lane whose
            // second column lies past the row reads the pair ending at its first
            const dv2 v = bload2(ru, rowok && ok0 ? (rowoff + (ok1 ? c0 : c0 - 1)) * 8u : kOOB);
            v0[i] = ok1 ? v.x : v.y;
            v1[i] = ok1 ? v.y : 0.0;
        }
        vh[i] = bload(ru, rowok && okh ? (rowoff + ch) * 8u : kOOB);
    }

    // spare LDS slots take the halo value of lanes without a halo column
    const int hidx = lane < P ? lane : (lane < 2 * P ? SW + lane : SW + 2 * P + (lane & 1));

    // 3. x pass, ring, y pass, stores
    const auto ro = buf(g.out, (size_t)X.R * Y.R);
    const auto rm = buf(g.omass, (MODE & kMass) ? (size_t)X.R * Y.R : 0);
    const auto rf = buf(g.farr, (MODE & kFarr) ? (size_t)X.R * Y.R : 0);
    const bool okc0 = xr0 < X.R, okc1 = xr1 < X.R;
    double ra0[W], rb0[W], ra1[W], rb1[W];
    double ymu[W], ydu[W];   // YIN: every row of the chunk interior, one row of y taps
    if constexpr (YIN) {
        const cdp um = (cdp)(Y.M + (size_t)Y.ilo * W), ud = (cdp)(Y.D + (size_t)Y.ilo * W);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            ymu[k] = um[k];
            ydu[k] = ud[k];
        }
    }
    if constexpr (kDma) {
        if constexpr (kCy) {
#pragma unroll
            for (int c = 0; c < NCV; ++c) cy[lane + 64 * c] = cv[c];
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): every row is in LDS
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        // 2. row i into LDS as soon as its loads are in (later rows keep loading while
        //    this one is computed and stored); LDS operations of one wave execute in
        //    order, the fence only keeps the compiler from reordering them
        if constexpr (!kDma) {
            rb[i][P + 2 * lane] = v0[i];
            rb[i][P + 2 * lane + 1] = v1[i];
        }
        rb[i][hidx] = vh[i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double t[2 * P + 2];
#pragma unroll
        for (int q = 0; q < 2 * P + 2; ++q) t[q] = rb[i][2 * lane + q];
        double a0 = 0.0, b0 = 0.0, a1 = 0.0, b1 = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            a0 = fma(m0[k], t[k], a0);
            b0 = fma(d0[k], t[k], b0);
            a1 = fma(m1[k], t[k + 1], a1);
            b1 = fma(d1[k], t[k + 1], b1);
        }
        ra0[i % W] = a0;
        rb0[i % W] = b0;
        ra1[i % W] = a1;
        rb1[i % W] = b1;
        if (i >= 2 * P) {
            const int j = i - 2 * P;   // output row y0 + j uses input rows j .. j + 2P
            const double* cr = &cy[j * CW];
            double ms0 = 0.0, ly0 = 0.0, lx0 = 0.0, ms1 = 0.0, ly1 = 0.0, lx1 = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                double my, dy;
                if constexpr (YIN) {
                    my = ymu[k];
                    dy = ydu[k];
                } else {
                    my = cr[k];
                    dy = cr[W + k];
                }
                const int sl = (j + k) % W;
                ms0 = fma(my, ra0[sl], ms0);
                ly0 = fma(dy, ra0[sl], ly0);
                lx0 = fma(my, rb0[sl], lx0);
                ms1 = fma(my, ra1[sl], ms1);
                ly1 = fma(dy, ra1[sl], ly1);
                lx1 = fma(my, rb1[sl], lx1);
            }
            const bool rowok = y0 + j < Y.R;
            const unsigned ob = (unsigned)((y0 + j) * X.R + xr0) * 8u;
            const unsigned o0 = rowok && okc0 ? ob : kOOB;
            const unsigned o1 = rowok && okc1 ? ob + 8u : kOOB;
            if constexpr ((MODE & kMass) != 0) {
                if constexpr (VEC) {
                    bstore2<kStream>(rm, o0, ms0, ms1);
                } else {
                    bstore<kStream>(rm, o0, ms0);
                    bstore<kStream>(rm, o1, ms1);
                }
            }
            double w0 = fma(g.alpha, ms0, g.beta * (lx0 + ly0));
            double w1 = fma(g.alpha, ms1, g.beta * (lx1 + ly1));
            if constexpr ((MODE & kScaleSrc) != 0) {
                w0 = fma(g.gsep, fx0 * cr[2 * W + 1], w0);
                w1 = fma(g.gsep, fx1 * cr[2 * W + 1], w1);
            }
            if constexpr ((MODE & kFarr) != 0) {
                if constexpr (VEC) {
                    const dv2 f = bload2(rf, o0);
                    w0 = fma(g.garr, f.x, w0);
                    w1 = fma(g.garr, f.y, w1);
                } else {
                    w0 = fma(g.garr, bload(rf, o0), w0);
                    w1 = fma(g.garr, bload(rf, o1), w1);
                }
            }
            if constexpr ((MODE & kScaleSrc) != 0) {
                w0 *= sx0 * cr[2 * W];
                w1 *= sx1 * cr[2 * W];
            }
            if constexpr (VEC) {
                bstore2<kStream>(ro, o0, w0, w1);
            } else {
                bstore<kStream>(ro, o0, w0);
                bstore<kStream>(ro, o1, w1);
            }
        }
    }
}

// The same chunk with one column per lane: a strip of 64 output columns, 8-byte accesses.
// Twice the waves for the same rows, each with half the arithmetic; the sums are formed
// in the same order, so both strip widths give the same bits.
template <int P, int TY>
struct Chunk2D1 {
    static constexpr int W = 2 * P + 1;
    static constexpr int NR = TY + 2 * P;
    static constexpr int SW = 64;
    static constexpr int RBW = SW + 2 * P + 2;
    static constexpr int CW = 2 * W + 2;
    static constexpr int NCV = (TY * CW + 63) / 64;
    static constexpr int LDS = NR * RBW + NCV * 64;
};

template <int P, int TY, int MODE>
__device__ __forceinline__ void apply2d_chunk1(const ApplyArgs& g, int bx, int by, double* lds)
{
    using C = Chunk2D1<P, TY>;
    constexpr int W = C::W, NR = C::NR, SW = C::SW, RBW = C::RBW, CW = C::CW, NCV = C::NCV;
    double (*rb)[RBW] = reinterpret_cast<double (*)[RBW]>(lds);
    double* cy = lds + NR * RBW;
    const AxisOp &X = g.ax[0], &Y = g.ax[1];
    const int x0 = bx * SW, y0 = by * TY;
    const int lane = threadIdx.x;
    const int Nx = X.N, Ny = Y.N;
    const int c0 = x0 + lane;
    const auto rxm = buf(X.M, (size_t)X.R * W), rxd = buf(X.D, (size_t)X.R * W);
    double m0[W], d0[W];
    if (x0 >= X.ilo && x0 + SW - 1 <= X.ihi) {   // interior strip: one row, uniform loads
        const cdp um = (cdp)(X.M + (size_t)X.ilo * W), ud = (cdp)(X.D + (size_t)X.ilo * W);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            m0[k] = um[k];
            d0[k] = ud[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            m0[k] = bload(rxm, c0 < X.R ? (unsigned)(c0 * W + k) * 8u : kOOB);
            d0[k] = bload(rxd, c0 < X.R ? (unsigned)(c0 * W + k) * 8u : kOOB);
        }
    }
    double sx0 = 1.0, fx0 = 1.0;
    if constexpr ((MODE & kScaleSrc) != 0) {
        const auto rxs = buf(X.S, X.R), rxf = buf(X.F, X.R);
        sx0 = bload(rxs, c0 < X.R ? (unsigned)c0 * 8u : kOOB);
        fx0 = bload(rxf, c0 < X.R ? (unsigned)c0 * 8u : kOOB);
    }
    {
        const auto rym = buf(Y.M, (size_t)Y.R * W), ryd = buf(Y.D, (size_t)Y.R * W);
        const auto rys = buf(Y.S, Y.R), ryf = buf(Y.F, Y.R);
        double cv[NCV];
#pragma unroll
        for (int c = 0; c < NCV; ++c) {
            const int i = lane + 64 * c;
            const int j = i / CW, k = i - j * CW;
            const int yr = y0 + j;
            const bool ok = i < TY * CW && yr < Y.R;
            const unsigned om = ok && k < W ? (unsigned)(yr * W + k) * 8u : kOOB;
            const unsigned od = ok && k >= W && k < 2 * W ? (unsigned)(yr * W + k - W) * 8u : kOOB;
            const unsigned os = ok && k == 2 * W ? (unsigned)yr * 8u : kOOB;
            const unsigned of = ok && k == 2 * W + 1 ? (unsigned)yr * 8u : kOOB;
            cv[c] = bload(rym, om) + bload(ryd, od) + bload(rys, os) + bload(ryf, of);
        }
#pragma unroll
        for (int c = 0; c < NCV; ++c) cy[lane + 64 * c] = cv[c];
    }
    const auto ru = buf(g.u, (size_t)Nx * Ny);
    const int ch = lane < P ? x0 - P + lane : x0 + SW + lane - P;
    const bool ok0 = c0 < Nx, okh = lane < 2 * P && ch >= 0 && ch < Nx;
    double v0[NR], vh[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int yi = y0 - P + i;
        const bool rowok = yi >= 0 && yi < Ny;
        const unsigned rowoff = (unsigned)yi * (unsigned)Nx;
        v0[i] = bload(ru, rowok && ok0 ? (rowoff + c0) * 8u : kOOB);
        vh[i] = bload(ru, rowok && okh ? (rowoff + ch) * 8u : kOOB);
    }
    const int hidx = lane < P ? lane : (lane < 2 * P ? SW + lane : SW + 2 * P + (lane & 1));
    const auto ro = buf(g.out, (size_t)X.R * Y.R);
    const auto rm = buf(g.omass, (MODE & kMass) ? (size_t)X.R * Y.R : 0);
    const auto rf = buf(g.farr, (MODE & kFarr) ? (size_t)X.R * Y.R : 0);
    const bool okc0 = c0 < X.R;
    double ra0[W], rb0[W];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        rb[i][P + lane] = v0[i];
        rb[i][hidx] = vh[i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double t[W];
#pragma unroll
        for (int q = 0; q < W; ++q) t[q] = rb[i][lane + q];
        double a0 = 0.0, b0 = 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            a0 = fma(m0[k], t[k], a0);
            b0 = fma(d0[k], t[k], b0);
        }
        ra0[i % W] = a0;
        rb0[i % W] = b0;
        if (i >= 2 * P) {
            const int j = i - 2 * P;
            const double* cr = &cy[j * CW];
            double ms0 = 0.0, ly0 = 0.0, lx0 = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const double my = cr[k], dy = cr[W + k];
                const int sl = (j + k) % W;
                ms0 = fma(my, ra0[sl], ms0);
                ly0 = fma(dy, ra0[sl], ly0);
                lx0 = fma(my, rb0[sl], lx0);
            }
            const bool rowok = y0 + j < Y.R;
            const unsigned o0 = rowok && okc0 ? (unsigned)((y0 + j) * X.R + c0) * 8u : kOOB;
            if constexpr ((MODE & kMass) != 0) bstore<kStream>(rm, o0, ms0);
            double w0 = fma(g.alpha, ms0, g.beta * (lx0 + ly0));
            if constexpr ((MODE & kScaleSrc) != 0) w0 = fma(g.gsep, fx0 * cr[2 * W + 1], w0);
            if constexpr ((MODE & kFarr) != 0) w0 = fma(g.garr, bload(rf, o0), w0);
            if constexpr ((MODE & kScaleSrc) != 0) w0 *= sx0 * cr[2 * W];
            bstore<kStream>(ro, o0, w0);
        }
    }
}

template <int P, int TY, int MODE>
__global__ __launch_bounds__(64) void apply2d1_kernel(ApplyArgs g, TileGrid tg)
{
    __shared__ __attribute__((aligned(16))) double lds[Chunk2D1<P, TY>::LDS];
    const int L = tg.TZ == 2 ? (int)blockIdx.x : xcd_logical_block(blockIdx.x, tg.nblk);
    const int bx = tg.TZ == 1 ? L / tg.ty : L % tg.tx;
    const int by = tg.TZ == 1 ? L % tg.ty : L / tg.tx;
    apply2d_chunk1<P, TY, MODE>(g, bx, by, lds);
}

template <int P, int TY, int MODE, bool VEC>
__global__ __launch_bounds__(64) void apply2d_kernel(ApplyArgs g, TileGrid tg)
{
    __shared__ __attribute__((aligned(16))) double lds[Chunk2D<P, TY>::LDS];
    // tg.TZ selects the block order (tuning): 0 = XCD-aware, row bands consecutive;
    // 1 = XCD-aware, strips consecutive; 2 = dispatch order, row bands consecutive
    const int L = tg.TZ == 2 ? (int)blockIdx.x : xcd_logical_block(blockIdx.x, tg.nblk);
    const int bx = tg.TZ == 1 ? L / tg.ty : L % tg.tx;
    const int by = tg.TZ == 1 ? L % tg.ty : L / tg.tx;
    if (by * TY >= g.ax[1].ilo && by * TY + TY - 1 <= g.ax[1].ihi)   // rows all interior
        apply2d_chunk<P, TY, MODE, VEC, true, true>(g, bx, by, lds);
    else
        apply2d_chunk<P, TY, MODE, VEC, true, false>(g, bx, by, lds);
}

// Rows without a u-term: out_r = S(r) ( gsep prod_a F_a(r_a) + garr farr_r ).
template <int MODE>
__global__ void rows_only_kernel(ApplyArgs g, int dim, size_t nrows)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows) return;
    const int rx = (int)(idx % g.ax[0].R);
    const int ry = dim > 1 ? (int)((idx / g.ax[0].R) % g.ax[1].R) : 0;
    const int rz = dim > 2 ? (int)(idx / ((size_t)g.ax[0].R * g.ax[1].R)) : 0;
    double s = g.ax[0].S[rx], f = g.ax[0].F[rx];
    if (dim > 1) { s *= g.ax[1].S[ry]; f *= g.ax[1].F[ry]; }
    if (dim > 2) { s *= g.ax[2].S[rz]; f *= g.ax[2].F[rz]; }
    finish_row<MODE>(g, idx, 0.0, 0.0, s, f);
}

// The same rows on a (x blocks, R_y, z groups of kRowsZ) grid: no index division per
// row; axes beyond the dimension have one row and tables of ones.  Products in the order
// of the kernel above, so both give the same bits.
constexpr int kRowsZ = 8;

template <int MODE>
__global__ void rows_only_grid_kernel(ApplyArgs g)
{
    const AxisOp &X = g.ax[0], &Y = g.ax[1], &Z = g.ax[2];
    const int ry = blockIdx.y;
    const double ys = Y.S[ry], yf = Y.F[ry];
    const int z1 = min(Z.R, (int)(blockIdx.z + 1) * kRowsZ);
    for (int rz = blockIdx.z * kRowsZ; rz < z1; ++rz) {
        const double zs = Z.S[rz], zf = Z.F[rz];
        const size_t row0 = ((size_t)rz * Y.R + ry) * X.R;
        for (int rx = blockIdx.x * blockDim.x + threadIdx.x; rx < X.R; rx += gridDim.x * blockDim.x) {
            double s = X.S[rx], f = X.F[rx];
            s *= ys;
            f *= yf;
            s *= zs;
            f *= zf;
            finish_row<MODE>(g, row0 + rx, 0.0, 0.0, s, f);
        }
    }
}

__global__ void copy_kernel(double* __restrict__ dst, const double* __restrict__ src, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// The memory traffic of the fused apply without its arithmetic: every value of src read
// once, written to two arrays, 16 bytes per lane and access, outputs streamed past the
// caches as the 2D kernel stores them.  A bandwidth reference, not part of the method.
__global__ __launch_bounds__(kBlock) void copy2_kernel(const double* __restrict__ src, double* __restrict__ a,
                                                       double* __restrict__ b, size_t n)
{
    const size_t i = 2 * ((size_t)blockIdx.x * kBlock + threadIdx.x);
    const auto rs = buf(src, n), ra = buf(a, n), rb = buf(b, n);
    if (i + 1 < n) {
        const dv2 v = bload2(rs, (unsigned)(i * 8));
        bstore2<kStream>(ra, (unsigned)(i * 8), v.x, v.y);
        bstore2<kStream>(rb, (unsigned)(i * 8), v.x, v.y);
    } else if (i < n) {
        const double v = bload(rs, (unsigned)(i * 8));
        bstore<kStream>(ra, (unsigned)(i * 8), v);
        bstore<kStream>(rb, (unsigned)(i * 8), v);
    }
}

}  // namespace iga
