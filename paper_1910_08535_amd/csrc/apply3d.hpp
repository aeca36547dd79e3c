// apply3d.hpp -- 3D rows by sum factorization with the z pass first:
//   z pass: Z1 = Mz u,  Z2 = Dz u
//   y pass: Y1 = My Z1, Y2 = Dy Z1 + My Z2
//   x pass: mass = Mx Y1, lap = Dx Y1 + Mx Y2
// (the same Kronecker factors as the 2D kernel, applied in another order; an exact
// re-association of the Gauss sums, so results agree with any other order to round-off).
//
// A workgroup owns an output tile of TX x TY rows of every plane of a z-chunk of TZ
// planes and streams through the chunk plane by plane:
//   * every thread owns a fixed set of (x, y) points of the tile's input footprint (the
//     tile plus p-wide halos, clipped to the array); their coefficients of the last 2p+1
//     planes sit in a register ring, so each coefficient is loaded once per chunk and the
//     z-halo planes cost loads only, never arithmetic;
//   * the z pass writes Z1, Z2 of the footprint to LDS; the y pass (two output rows per
//     task, so 2p+2 loads feed 2 outputs) writes Y1, Y2 to LDS; the x pass (two output
//     columns per task, 128-bit LDS reads) forms the rows and stores them;
//   * tasks are enumerated flat over the tile, so tiles of any width keep the lanes busy.
// Band entries: rows of the interior range of an axis share one set of taps, which every
// thread holds once (uniform loads); only the few tasks that touch the first or last 2p
// rows of an axis read their own rows' taps.  Taps of the z pass are uniform per plane.
#pragma once

#include "apply.hpp"
#include "common.hpp"

namespace iga {

// Launch geometry of apply3d_kernel.
struct Plan3D {
    int tx, ty, tz, nblk;   // tiles along x, y and z-chunks; their product
    int TX, TY, TZ;         // output rows per tile along x (even), y, z
    int LW;                 // LDS row length: TX + 2p (even)
};

// footprint points per thread (z pass): the register ring holds (2p+1) x npz values
__host__ __device__ constexpr int npz(int P)
{
    return P == 3 ? 2 : 3;
}
constexpr int kMaxNT3 = 512;   // threads per workgroup, at most

// LDS of a plan.  Z1, Z2 are stored by column (LW columns of zcol(TY, P) doubles: the
// footprint's TY + 2p rows, padded to an odd count so that lanes reading neighbouring
// columns hit different banks) -- the y pass then reads consecutive addresses; Y1, Y2
// are stored by row (TY rows of LW doubles) for the x pass.
__host__ __device__ inline int zcol(int TY, int P)
{
    return (TY + 2 * P) | 1;
}

// After them, staged once per workgroup: the band rows of the tile's x columns and y
// rows ([M (2p+1) | D (2p+1)] each; read only by tasks on the first or last 2p rows of
// an axis) and their S and F factors.  The plane loop then issues no global loads besides
// the coefficient prefetch, so no memory wait in it drains that prefetch.
__host__ __device__ inline size_t lds3d_doubles(int TX, int TY, int LW, int P)
{
    return (size_t)(2 * zcol(TY, P) + 2 * TY) * (size_t)LW + (size_t)(TX + TY) * (4 * P + 2) +
           2 * (size_t)(TX + TY);
}

// Band rows r0 .. r0+n-1 of an axis into LDS rows of 2W doubles (rows past the axis: 0).
template <int W>
__device__ __forceinline__ void stage_taps(double* dst, const AxisOp& A, int r0, int n, int tid, int NT)
{
    for (int i = tid; i < n * 2 * W; i += NT) {
        const int j = i / (2 * W), k = i - j * (2 * W);
        const int r = r0 + j;
        double v = 0.0;
        if (r < A.R) v = k < W ? A.M[(size_t)r * W + k] : A.D[(size_t)r * W + k - W];
        dst[i] = v;
    }
}

template <int W>
__device__ __forceinline__ void lds_taps(double (&m)[W], double (&d)[W], const double* row)
{
#pragma unroll
    for (int k = 0; k < W; ++k) {
        m[k] = row[k];
        d[k] = row[W + k];
    }
}

// Unaligned (8-byte) pair of doubles: one 16-byte store where the hardware allows it.
typedef double dv2u __attribute__((ext_vector_type(2), aligned(8)));

// Loads through the constant address space: with a uniform address the compiler issues
// scalar loads, and the taps then occupy scalar registers instead of vector ones.
typedef const __attribute__((address_space(4))) double* cdptr;

template <int W>
__device__ __forceinline__ void uniform_row(double (&m)[W], double (&d)[W], const double* M,
                                            const double* D, int row)
{
    const cdptr pm = (cdptr)(M + (size_t)row * W);
    const cdptr pd = (cdptr)(D + (size_t)row * W);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        m[k] = pm[k];
        d[k] = pd[k];
    }
}

// A row index the compiler cannot see through: the taps loaded with it are re-read in
// the pass that uses them (scalar loads hitting the scalar cache) instead of being kept
// live across the whole plane loop, which would need more scalar registers than exist.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// One output of a pass: a stencil over a[o .. o+2P] (first factor) and b[] (second).
template <int P>
__device__ __forceinline__ void pstep(const double (&a)[2 * P + 2], const double (&b)[2 * P + 2], int o,
                                      const double (&m)[2 * P + 1], const double (&d)[2 * P + 1],
                                      double& y1, double& y2)
{
    y1 = y2 = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * P + 1; ++k) {
        y1 = fma(m[k], a[k + o], y1);
        y2 = fma(d[k], a[k + o], y2);
        y2 = fma(m[k], b[k + o], y2);
    }
}

// y pass of one task: output rows r and r+1 from the 2P+2 values a[], b[] of Z1, Z2 in
// the column (input rows r-P .. r+P+1).
template <int P>
__device__ __forceinline__ void ypair(const double (&a)[2 * P + 2], const double (&b)[2 * P + 2],
                                      const double (&m0)[2 * P + 1], const double (&d0)[2 * P + 1],
                                      const double (&m1)[2 * P + 1], const double (&d1)[2 * P + 1],
                                      double& y10, double& y20, double& y11, double& y21)
{
    y10 = y20 = y11 = y21 = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * P + 1; ++k) {
        y10 = fma(m0[k], a[k], y10);
        y20 = fma(d0[k], a[k], y20);
        y20 = fma(m0[k], b[k], y20);
        y11 = fma(m1[k], a[k + 1], y11);
        y21 = fma(d1[k], a[k + 1], y21);
        y21 = fma(m1[k], b[k + 1], y21);
    }
}

template <int P, int MODE>
__global__ __launch_bounds__(kMaxNT3, 4) void apply3d_kernel(ApplyArgs g, Plan3D pl)
{
    constexpr int W = 2 * P + 1;
    constexpr int kNPZ = npz(P);
    extern __shared__ __attribute__((aligned(16))) double lds3[];
    const AxisOp &X = g.ax[0], &Y = g.ax[1], &Z = g.ax[2];
    const int NT = (int)blockDim.x, tid = (int)threadIdx.x;
    const int L = xcd_logical_block((int)blockIdx.x, pl.nblk);
    const int bx = L % pl.tx, by = (L / pl.tx) % pl.ty, bz = L / (pl.tx * pl.ty);
    const int x0 = bx * pl.TX, y0 = by * pl.TY, z0 = bz * pl.TZ;
    const int x1 = min(x0 + pl.TX, X.R), y1 = min(y0 + pl.TY, Y.R), z1 = min(z0 + pl.TZ, Z.R);
    if (x0 >= x1 || y0 >= y1 || z0 >= z1) return;   // the whole workgroup
    const int LW = pl.LW, LH = zcol(pl.TY, P);
    double* sZ1 = lds3;                 // [LW][LH]: column-major
    double* sZ2 = sZ1 + LH * LW;
    double* sY1 = sZ2 + LH * LW;        // [TY][LW]: row-major
    double* sY2 = sY1 + pl.TY * LW;

    // band rows of the tile's columns and rows, then their S and F: [x S | x F | y S | y F]
    double* tx_ = sY2 + pl.TY * LW;
    double* ty_ = tx_ + pl.TX * 2 * W;
    double* sfx = ty_ + pl.TY * 2 * W;
    double* sfy = sfx + 2 * pl.TX;
    stage_taps<W>(tx_, X, x0, pl.TX, tid, NT);
    stage_taps<W>(ty_, Y, y0, pl.TY, tid, NT);

    // LDS slots outside the array stay zero for the whole chunk
    const int nl = (2 * LH + 2 * pl.TY) * LW;
    for (int i = tid; i < nl; i += NT) lds3[i] = 0.0;
    if constexpr ((MODE & kScaleSrc) != 0) {
        for (int i = tid; i < pl.TX; i += NT) {
            const int x = min(x0 + i, X.R - 1);
            sfx[i] = X.S[x];
            sfx[pl.TX + i] = X.F[x];
        }
        for (int i = tid; i < pl.TY; i += NT) {
            const int y = min(y0 + i, Y.R - 1);
            sfy[i] = Y.S[y];
            sfy[pl.TY + i] = Y.F[y];
        }
    }

    // footprint of the tile: input columns xa..xb-1 and rows ya..yb-1
    const int NX = X.N, NY = Y.N, NZ = Z.N;
    const int xa = max(x0 - P, 0), xb = min(x1 + P, NX);
    const int ya = max(y0 - P, 0), yb = min(y1 + P, NY);
    const int RW = xb - xa, npt = RW * (yb - ya);
    unsigned goff[kNPZ];
    int loff[kNPZ];
#pragma unroll
    for (int i = 0; i < kNPZ; ++i) {
        const int j = tid + i * NT;
        const int r = j / RW, cc = j - r * RW;
        const bool ok = j < npt;
        goff[i] = ok ? (unsigned)((ya + r) * NX + xa + cc) * 8u : kOOB;
        loff[i] = ok ? (xa + cc - (x0 - P)) * LH + (ya + r - (y0 - P)) : -1;
    }
    const size_t plane = (size_t)NX * NY;
    auto plane_buf = [&](int zi) {
        const bool ok = zi >= 0 && zi < NZ;
        return buf(g.u + (ok ? (size_t)zi * plane : 0), ok ? plane : 0);
    };

    // ring: plane z0 - P + s in slot s (mod W); slot 2P is loaded last
    double rz[W][kNPZ];
#pragma unroll
    for (int s = 0; s < W; ++s) {
        const auto rb = plane_buf(z0 - P + s);
#pragma unroll
        for (int i = 0; i < kNPZ; ++i) rz[s][i] = bload(rb, goff[i]);
    }
    __syncthreads();   // LDS zeroed before the first footprint write

    // task counts of the y and x passes
    const int TYv = y1 - y0, TXv = x1 - x0;
    const int npy = (TYv + 1) >> 1;
    const int npx = (TXv + 1) >> 1;
    int ia = X.ilo - x0;
    ia = ia <= 0 ? 0 : (ia + 1) >> 1;                  // first pair with x0 + 2i >= ilo
    int ib = X.ihi - x0 - 1;
    ib = ib < 0 ? 0 : (ib >> 1) + 1;                   // pairs with x0 + 2i + 1 <= ihi
    ia = min(ia, npx);
    ib = min(max(ib, ia), npx);
    const int nI = ib - ia, nB = npx - nI;
    const int ntxI = TYv * nI, ntx = TYv * npx;
    const int lc0 = xa - (x0 - P);   // LDS column of input column xa
    // strides of the division-free task walks (NT tasks per step)
    const int ydq = NT / RW, ydc = NT - (NT / RW) * RW;
    const int xdr = nI > 0 ? NT / nI : 0, xdi = nI > 0 ? NT - (NT / nI) * nI : 0;

    int cur = 0;   // slot of plane zo - P
    for (int zo = z0; zo < z1; ++zo) {
        // ---- z pass (slot layout known at compile time in each branch) ----
        double zm[W], zd[W];
        uniform_row<W>(zm, zd, Z.M, Z.D, opaque(zo));
#pragma unroll
        for (int ph = 0; ph < W; ++ph) {
            if (ph == cur) {
#pragma unroll
                for (int i = 0; i < kNPZ; ++i) {
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const double v = rz[(ph + k) % W][i];
                        s1 = fma(zm[k], v, s1);
                        s2 = fma(zd[k], v, s2);
                    }
                    if (loff[i] >= 0) {
                        sZ1[loff[i]] = s1;
                        sZ2[loff[i]] = s2;
                    }
                }
                // plane zo - P is no longer needed: its slot takes plane zo + P + 1
                const auto rb = plane_buf(zo + P + 1 < z1 + P ? zo + P + 1 : -1);
#pragma unroll
                for (int i = 0; i < kNPZ; ++i) rz[ph][i] = bload(rb, goff[i]);
            }
        }
        cur = cur == W - 1 ? 0 : cur + 1;
        __syncthreads();

        // ---- y pass: rows y0 + 2q, y0 + 2q + 1 of footprint column xa + c ----
        double yim[W], yid[W];
        uniform_row<W>(yim, yid, Y.M, Y.D, opaque(Y.ilo <= Y.ihi ? Y.ilo : 0));
        // task t = q * RW + c, walked without divisions
        int q = tid / RW, c = tid - (tid / RW) * RW;
        for (; q < npy;) {
            const int r0 = y0 + 2 * q;
            const int lc = lc0 + c;
            const double* z1p = sZ1 + lc * LH + 2 * q;   // input rows r0 - P .. r0 + P + 1
            const double* z2p = sZ2 + lc * LH + 2 * q;
            double a[2 * P + 2], b[2 * P + 2];
#pragma unroll
            for (int k = 0; k < 2 * P + 2; ++k) {
                a[k] = z1p[k];
                b[k] = z2p[k];
            }
            double y10, y20, y11, y21;
            if (r0 >= Y.ilo && r0 + 1 <= Y.ihi) {
                ypair<P>(a, b, yim, yid, yim, yid, y10, y20, y11, y21);
            } else {
                double m[W], d[W];
                lds_taps<W>(m, d, ty_ + (2 * q) * 2 * W);
                pstep<P>(a, b, 0, m, d, y10, y20);
                lds_taps<W>(m, d, ty_ + (2 * q + 1) * 2 * W);
                pstep<P>(a, b, 1, m, d, y11, y21);
            }
            sY1[(2 * q) * LW + lc] = y10;
            sY2[(2 * q) * LW + lc] = y20;
            if (r0 + 1 < y1) {
                sY1[(2 * q + 1) * LW + lc] = y11;
                sY2[(2 * q + 1) * LW + lc] = y21;
            }
            c += ydc;
            q += ydq;
            if (c >= RW) {
                c -= RW;
                ++q;
            }
        }
        __syncthreads();

        // ---- x pass: columns x0 + 2i, x0 + 2i + 1 of row y; interior pairs first ----
        const int oz = zo;
        const double sz = Z.S[oz], fz = Z.F[oz];
        double xim[W], xid[W];
        uniform_row<W>(xim, xid, X.M, X.D, opaque(X.ilo <= X.ihi ? X.ilo : 0));
        // interior tasks t = row * nI + ii, walked without divisions
        int irow = 0, ii = 0;
        if (nI > 0) {
            irow = tid / nI;
            ii = tid - irow * nI;
        }
        for (int t = tid; t < ntx; t += NT) {
            int row, i;
            bool inner;
            if (t < ntxI) {
                row = irow;
                i = ia + ii;
                inner = true;
            } else {
                const int b = t - ntxI;
                row = b / nB;
                const int j = b - row * nB;
                i = j < ia ? j : j + nI;
                inner = false;
            }
            // LDS positions 2i .. 2i + 2P + 1 hold input columns x0 + 2i - P ..
            const dv2* p1 = reinterpret_cast<const dv2*>(sY1 + row * LW + 2 * i);
            const dv2* p2 = reinterpret_cast<const dv2*>(sY2 + row * LW + 2 * i);
            double a[2 * P + 2], b[2 * P + 2];
#pragma unroll
            for (int k = 0; k < P + 1; ++k) {
                const dv2 va = p1[k], vb = p2[k];
                a[2 * k] = va.x;
                a[2 * k + 1] = va.y;
                b[2 * k] = vb.x;
                b[2 * k + 1] = vb.y;
            }
            double ms0, lp0, ms1, lp1;
            const int gx = x0 + 2 * i, gy = y0 + row;
            if (inner) {
                ypair<P>(a, b, xim, xid, xim, xid, ms0, lp0, ms1, lp1);
            } else {
                double m[W], d[W];
                lds_taps<W>(m, d, tx_ + (2 * i) * 2 * W);
                pstep<P>(a, b, 0, m, d, ms0, lp0);
                lds_taps<W>(m, d, tx_ + (2 * i + 1) * 2 * W);
                pstep<P>(a, b, 1, m, d, ms1, lp1);
            }
            const size_t idx = ((size_t)oz * Y.R + gy) * X.R + gx;
            double s0 = 1.0, s1 = 1.0, f0 = 1.0, f1 = 1.0;
            if constexpr ((MODE & kScaleSrc) != 0) {
                const double syz = sfy[row] * sz, fyz = sfy[pl.TY + row] * fz;
                s0 = sfx[2 * i] * syz;
                f0 = sfx[pl.TX + 2 * i] * fyz;
                s1 = sfx[2 * i + 1] * syz;
                f1 = sfx[pl.TX + 2 * i + 1] * fyz;
            }
            finish_pair<MODE>(g, idx, ms0, lp0, s0, f0, ms1, lp1, s1, f1, gx + 1 < x1);
            ii += xdi;
            irow += xdr;
            if (ii >= nI) {
                ii -= nI;
                ++irow;
            }
        }
    }
}

}  // namespace iga
