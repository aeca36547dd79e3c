// apply3d.hpp -- 3D rows by sum factorization with the z pass first:
//   z pass: Z1 = Mz u,  Z2 = Dz u
//   y pass: Y1 = My Z1, Y2 = Dy Z1 + My Z2
//   x pass: mass = Mx Y1, lap = Dx Y1 + Mx Y2
// (the same Kronecker factors as the 2D kernel, applied in another order; an exact
// re-association of the Gauss sums, so results agree with any other order to round-off).
//
// A workgroup owns an output tile of TX x TY rows of every plane of a z-chunk of TZ
// planes and streams through the chunk plane by plane:
//   * the three passes are software-pipelined over the planes: step k runs the z pass of
//     plane k (registers -> LDS stage Z), the y pass of plane k-1 (stage Z -> stage Y) and
//     the x pass of plane k-2 (stage Y -> memory), each stage double-buffered, so a plane
//     costs ONE workgroup barrier and the work of three planes is in flight together;
//   * each wave has one role for the whole chunk (Roles3D): the first waves run the z
//     pass, the next the y pass, the last the x pass, each role in a loop of its own with
//     the same steps and barriers.  The passes of one step then run side by side on
//     different waves instead of one after the other in every wave, each role keeps only
//     its own registers live, and only the z waves load and only the x waves store;
//   * a z thread owns fixed (x, y) points of the tile's input footprint (the tile plus
//     p-wide halos, clipped to the array); their coefficients of the planes zo-p .. zo+p
//     sit in a register ring (2p slots rotating, the newest plane in its own register), so
//     each coefficient is loaded once per chunk and the z-halo planes cost loads only;
//   * a y task is two output rows of one footprint column, from the 2p + 2 values of that
//     column (stage Z is stored by columns, an odd column stride keeping lanes on distinct
//     banks); an x task is two output columns of one row, from 128-bit reads of a stage Y
//     row, stored with one 16-byte access.  A thread's tasks are fixed for the whole chunk,
//     so their addresses are computed once;
//   * tasks of interior rows (columns) come first, padded to whole waves, so that each
//     wave takes one branch of the tap choice; interior taps are read with uniform
//     (scalar) loads once per step, the rows at the ends of an axis read their own taps,
//     staged in LDS once per workgroup.  Taps of the z pass are uniform per plane.
// Without mass output the y pass folds the operator weights into one array,
// B = alpha Y1 + beta Y2, so the x pass forms  alpha mass + beta lap = Mx B + beta Dx Y1
// with two stencils instead of three.
#pragma once

#include "apply.hpp"
#include "common.hpp"

namespace iga {

// Launch geometry of apply3d_kernel.
struct Plan3D {
    int tx, ty, tz, nblk;   // tiles along x, y and z-chunks; their product
    int TX, TY, TZ;         // output rows per tile along x (even), y, z
    int LW;                 // footprint columns: TX + 2p
    int LS;                 // row stride of the LDS stages: LW rounded up to even
    int LH;                 // footprint rows: TY + 2p
};

constexpr int kRY3 = 2;        // output rows per y task
constexpr int kMaxNT3 = 512;   // threads per workgroup, at most

// Waves of a workgroup by role: the first WZ waves run the z pass (NZ footprint points per
// thread), the next WY the y pass (up to NY tasks per thread), the last WX the x pass (up
// to NX tasks per thread).  Sized so that each role carries about the same arithmetic
// (for p = 3: 6 points x 14, 2 tasks x 42, 3 tasks x 28 FMAs per thread and step).
template <int P>
struct Roles3D {
    static constexpr int WZ = 3, NZ = 6, WY = 3, NY = P == 3 ? 2 : 3, WX = 2, NX = P == 3 ? 3 : 4;
    static_assert(WZ + WY + WX == kMaxNT3 / 64, "every wave has a role");
};

// Footprint points, y tasks and x tasks a workgroup can hold.
template <int P>
__host__ __device__ constexpr int z_cap3() { return Roles3D<P>::NZ * 64 * Roles3D<P>::WZ; }
template <int P>
__host__ __device__ constexpr int y_cap3() { return Roles3D<P>::NY * 64 * Roles3D<P>::WY; }
template <int P>
__host__ __device__ constexpr int x_cap3() { return Roles3D<P>::NX * 64 * Roles3D<P>::WX; }
__host__ __device__ constexpr int z_cap3(int P) { return P == 3 ? z_cap3<3>() : z_cap3<2>(); }
__host__ __device__ constexpr int y_cap3(int P) { return P == 3 ? y_cap3<3>() : y_cap3<2>(); }
__host__ __device__ constexpr int x_cap3(int P) { return P == 3 ? x_cap3<3>() : x_cap3<2>(); }

// LDS of a plan, in doubles: stage Z (two buffers of Z1 | Z2, LW columns of (LH | 1)),
// stage Y (two buffers of A | B, TY rows of LS), then, staged once per workgroup, the band rows
// of the tile's x columns and y rows ([M (2p+1) | D (2p+1)] each; read only by tasks on
// the first or last rows of an axis) and their S and F factors.
__host__ __device__ inline size_t lds3d_doubles(int TX, int TY, int LS, int LH, int P)
{
    const size_t zsz = (size_t)(LH | 1) * (TX + 2 * P);   // stage Z by columns
    return 4 * zsz + 4 * (size_t)TY * LS + (size_t)(TX + TY) * (4 * P + 2) + 2 * (size_t)(TX + TY);
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

// Loads through the constant address space (cdp, apply.hpp): with a uniform address the
// compiler issues scalar loads, and the taps then occupy scalar registers instead of
// vector ones.

template <int W>
__device__ __forceinline__ void uniform_row(double (&m)[W], double (&d)[W], const double* M,
                                            const double* D, int row)
{
    const cdp pm = (cdp)(M + (size_t)row * W);
    const cdp pd = (cdp)(D + (size_t)row * W);
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

// Rows idx and idx + 1 (the second only when `two`) from v = alpha mass + beta lap, with
// the epilogue of row_value (sources, then the scale) and one 16-byte store per pair.
template <int MODE>
__device__ __forceinline__ void finish_folded(const ApplyArgs& g, size_t idx, double v0, double s0, double f0,
                                              double v1, double s1, double f1, bool two)
{
    typedef double pair_t __attribute__((ext_vector_type(2), aligned(8)));
    double a0 = 0.0, a1 = 0.0;
    if constexpr ((MODE & kFarr) != 0) {
        if (two) {
            const pair_t fa = *reinterpret_cast<const pair_t*>(g.farr + idx);
            a0 = fa.x;
            a1 = fa.y;
        } else {
            a0 = g.farr[idx];
        }
    }
    if constexpr ((MODE & kScaleSrc) != 0) {
        v0 = fma(g.gsep, f0, v0);
        v1 = fma(g.gsep, f1, v1);
    }
    if constexpr ((MODE & kFarr) != 0) {
        v0 = fma(g.garr, a0, v0);
        v1 = fma(g.garr, a1, v1);
    }
    if constexpr ((MODE & kScaleSrc) != 0) {
        v0 *= s0;
        v1 *= s1;
    }
    if (two)
        *reinterpret_cast<pair_t*>(g.out + idx) = pair_t{v0, v1};
    else
        g.out[idx] = v0;
}

// One output of a pass: a stencil over a[o .. o+2P] (first factor) and b[] (second).
template <int P, int N>
__device__ __forceinline__ void pstep(const double (&a)[N], const double (&b)[N], int o,
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

// The x pass of one output column (offset o in the 2P + 2 values a[] (Y1) and b[] (Y2, or
// the folded B)).  Folded: o0 = Mx B, o1 = Dx Y1 (the row is alpha mass + beta lap =
// o0 + beta o1); otherwise o0 = mass, o1 = lap.
template <int P, bool FOLD>
__device__ __forceinline__ void xcol(const double (&a)[2 * P + 2], const double (&b)[2 * P + 2], int o,
                                     const double (&m)[2 * P + 1], const double (&d)[2 * P + 1], double& o0,
                                     double& o1)
{
    if constexpr (FOLD) {
        o0 = o1 = 0.0;
#pragma unroll
        for (int k = 0; k < 2 * P + 1; ++k) {
            o0 = fma(m[k], b[k + o], o0);
            o1 = fma(d[k], a[k + o], o1);
        }
    } else {
        pstep<P>(a, b, o, m, d, o0, o1);
    }
}

// Tile L (x fastest, then y, then z-chunk) of the plan, by a workgroup of kMaxNT3 threads
// with the plan's LDS bytes of dynamic shared memory.
template <int P, int MODE>
__device__ __forceinline__ void apply3d_tile(const ApplyArgs& g, const Plan3D& pl, int L)
{
    using RL = Roles3D<P>;
    constexpr int W = 2 * P + 1;
    constexpr int NZ = RL::NZ, NY = RL::NY, NX = RL::NX;
    constexpr int TZT = 64 * RL::WZ, TYT = 64 * RL::WY, TXT = 64 * RL::WX;   // threads per role
    constexpr bool kFold = (MODE & kMass) == 0;   // B = alpha Y1 + beta Y2
    extern __shared__ __attribute__((aligned(16))) double lds3[];
    const AxisOp &X = g.ax[0], &Y = g.ax[1], &Z = g.ax[2];
    const int tid = (int)threadIdx.x;
    const int bx = L % pl.tx, by = (L / pl.tx) % pl.ty, bz = L / (pl.tx * pl.ty);
    const int x0 = bx * pl.TX, y0 = by * pl.TY, z0 = bz * pl.TZ;
    const int x1 = min(x0 + pl.TX, X.R), y1 = min(y0 + pl.TY, Y.R), z1 = min(z0 + pl.TZ, Z.R);
    if (x0 >= x1 || y0 >= y1 || z0 >= z1) return;   // the whole workgroup
    const int LS = pl.LS, LH = pl.LH;
    const int LHc = LH | 1;             // column stride of stage Z (odd: no bank conflicts)
    const int zsz = LHc * pl.LW, ysz = pl.TY * LS;
    double* const sZ = lds3;            // [2 buffers][Z1 | Z2][LW columns][LHc]
    double* const sY = sZ + 4 * zsz;    // [2 buffers][A | B][TY][LS]
    double* const tx_ = sY + 4 * ysz;   // band rows of the tile's columns, then rows
    double* const ty_ = tx_ + pl.TX * 2 * W;
    double* const sfx = ty_ + pl.TY * 2 * W;   // [x S | x F | y S | y F]
    double* const sfy = sfx + 2 * pl.TX;
    stage_taps<W>(tx_, X, x0, pl.TX, tid, kMaxNT3);
    stage_taps<W>(ty_, Y, y0, pl.TY, tid, kMaxNT3);
    for (int i = tid; i < 4 * (zsz + ysz); i += kMaxNT3) lds3[i] = 0.0;
    for (int i = tid; i < pl.TX; i += kMaxNT3) {
        const int x = min(x0 + i, X.R - 1);
        sfx[i] = X.S[x];
        sfx[pl.TX + i] = X.F[x];
    }
    for (int i = tid; i < pl.TY; i += kMaxNT3) {
        const int y = min(y0 + i, Y.R - 1);
        sfy[i] = Y.S[y];
        sfy[pl.TY + i] = Y.F[y];
    }
    const int NX_ = X.N, NYc = Y.N, NZc = Z.N;
    const int xa = max(x0 - P, 0), xb = min(x1 + P, NX_);
    const int ya = max(y0 - P, 0), yb = min(y1 + P, NYc);
    const int RW = xb - xa, npt = RW * (yb - ya);
    const int lc0 = xa - (x0 - P);   // stage column of input column xa
    const int TYv = y1 - y0, TXv = x1 - x0, TZv = z1 - z0;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    __syncthreads();   // stages zeroed, taps and factors staged

    // Every role runs TZv + 2 steps with one barrier each: step k is the z pass of plane
    // z0 + k, the y pass of plane z0 + k - 1 and the x pass of plane z0 + k - 2.
    if (wave < RL::WZ) {
        // ---- z pass: footprint points j = tid + i TZT of this thread; their coefficients
        // of the planes zo-p .. zo+p in a register ring (2p slots rotating, the newest in nv)
        unsigned goff[NZ];
        int loff[NZ];
#pragma unroll
        for (int i = 0; i < NZ; ++i) {
            const int j = tid + i * TZT;
            const int r = j / RW, cc = j - r * RW;
            const bool ok = j < npt;
            goff[i] = ok ? (unsigned)((ya + r) * NX_ + xa + cc) * 8u : kOOB;
            loff[i] = ok ? (lc0 + cc) * LHc + (ya + r - (y0 - P)) : -1;
        }
        const size_t plane = (size_t)NX_ * NYc;
        auto plane_buf = [&](int zi) {
            const bool ok = zi >= 0 && zi < NZc && zi < z1 + P;
            return buf(g.u + (ok ? (size_t)zi * plane : 0), ok ? plane : 0);
        };
        double rz[2 * P][NZ], nv[NZ];
#pragma unroll
        for (int s2 = 0; s2 < 2 * P; ++s2) {
            const auto rb = plane_buf(z0 - P + s2);
#pragma unroll
            for (int i = 0; i < NZ; ++i) rz[s2][i] = bload(rb, goff[i]);
        }
        {
            const auto rb = plane_buf(z0 + P);
#pragma unroll
            for (int i = 0; i < NZ; ++i) nv[i] = bload(rb, goff[i]);
        }
        int cur = 0;   // ring slot of plane zo - P
        for (int k = 0; k < TZv + 2; ++k) {
            const int zo = min(z0 + k, z1 - 1);
            double* const z1s = sZ + (k & 1) * 2 * zsz;
            double* const z2s = z1s + zsz;
            double zm[W], zd[W];
            uniform_row<W>(zm, zd, Z.M, Z.D, opaque(zo));
#pragma unroll
            for (int ph = 0; ph < 2 * P; ++ph) {
                if (ph == cur) {
#pragma unroll
                    for (int i = 0; i < NZ; ++i) {
                        if (k < TZv && loff[i] >= 0) {   // the last two steps only rotate
                            double s1 = 0.0, s2 = 0.0;
#pragma unroll
                            for (int kk = 0; kk < 2 * P; ++kk) {
                                const double v = rz[(ph + kk) % (2 * P)][i];
                                s1 = fma(zm[kk], v, s1);
                                s2 = fma(zd[kk], v, s2);
                            }
                            s1 = fma(zm[2 * P], nv[i], s1);
                            s2 = fma(zd[2 * P], nv[i], s2);
                            z1s[loff[i]] = s1;
                            z2s[loff[i]] = s2;
                        }
                        rz[ph][i] = nv[i];   // plane zo - P leaves, plane zo + P takes its slot
                    }
                }
            }
            cur = cur == 2 * P - 1 ? 0 : cur + 1;
            const auto rb = plane_buf(z0 + k + P + 1);
#pragma unroll
            for (int i = 0; i < NZ; ++i) nv[i] = bload(rb, goff[i]);
            __syncthreads();
        }
    } else if (wave < RL::WZ + RL::WY) {
        // ---- y pass: tasks t = tid' + i TYT (two output rows 2q, 2q+1 of footprint column
        // c); tasks of interior row pairs first, padded to whole waves
        const int tyd = tid - TZT;
        const int nqy = (TYv + 1) >> 1;
        int qa = Y.ilo - y0;
        qa = qa <= 0 ? 0 : (qa + 1) >> 1;                  // first pair with y0 + 2q >= ilo
        int qb = Y.ihi - y0 - 1;
        qb = qb < 0 ? 0 : (qb >> 1) + 1;                   // pairs with y0 + 2q + 1 <= ihi
        qa = min(qa, nqy);
        qb = min(max(qb, qa), nqy);
        const int nYI = (qb - qa) * RW, nYIp = (nYI + 63) & ~63, nYB = (nqy - (qb - qa)) * RW;
        int tq[NY], tc[NY];   // pair q (flags in the high bits: interior, two rows, valid), column
#pragma unroll
        for (int i = 0; i < NY; ++i) {
            const int t = tyd + i * TYT;
            bool yv, yint;
            int yq, yc;
            if (t < nYIp) {
                yint = true;
                yv = t < nYI;
                const int u = yv ? t : 0;
                yq = qa + u / RW;
                yc = u - (u / RW) * RW;
            } else {
                yint = false;
                const int t0 = t - nYIp;
                yv = t0 < nYB;
                const int u = yv ? t0 : 0;
                const int j = u / RW;
                yq = j < qa ? j : j + (qb - qa);
                yc = u - j * RW;
            }
            const bool ytwo = 2 * yq + 1 < TYv;
            tq[i] = yq | (yint ? 1 << 16 : 0) | (ytwo ? 1 << 17 : 0) | (yv ? 1 << 18 : 0);
            tc[i] = lc0 + yc;
        }
        for (int k = 0; k < TZv + 2; ++k) {
            if (k >= 1 && k <= TZv) {
                double yim[W], yid[W];
                uniform_row<W>(yim, yid, Y.M, Y.D, opaque(Y.ilo <= Y.ihi ? Y.ilo : 0));
#pragma unroll
                for (int i = 0; i < NY; ++i) {
                    const int yq = tq[i] & 0xffff, ylc = tc[i];
                    if (!(tq[i] & (1 << 18))) continue;
                    const bool yint = (tq[i] & (1 << 16)) != 0, ytwo = (tq[i] & (1 << 17)) != 0;
                    const double* const c1 = sZ + ((k - 1) & 1) * 2 * zsz + ylc * LHc + 2 * yq;
                    const double* const c2 = c1 + zsz;
                    double* const ya_ = sY + ((k - 1) & 1) * 2 * ysz + 2 * yq * LS + ylc;
                    double* const yb_ = ya_ + ysz;
                    double y10 = 0.0, y20 = 0.0, y11 = 0.0, y21 = 0.0;
                    if (yint) {
#pragma unroll
                        for (int kk = 0; kk < 2 * P + 2; ++kk) {
                            const double av = c1[kk], bv = c2[kk];
                            if (kk <= 2 * P) {
                                y10 = fma(yim[kk], av, y10);
                                y20 = fma(yid[kk], av, y20);
                                y20 = fma(yim[kk], bv, y20);
                            }
                            if (kk >= 1) {
                                y11 = fma(yim[kk - 1], av, y11);
                                y21 = fma(yid[kk - 1], av, y21);
                                y21 = fma(yim[kk - 1], bv, y21);
                            }
                        }
                    } else {
                        double m[W], d[W];
                        lds_taps<W>(m, d, ty_ + (2 * yq) * 2 * W);
#pragma unroll
                        for (int kk = 0; kk < W; ++kk) {
                            const double av = c1[kk], bv = c2[kk];
                            y10 = fma(m[kk], av, y10);
                            y20 = fma(d[kk], av, y20);
                            y20 = fma(m[kk], bv, y20);
                        }
                        lds_taps<W>(m, d, ty_ + (2 * yq + 1) * 2 * W);
#pragma unroll
                        for (int kk = 0; kk < W; ++kk) {
                            const double av = c1[kk + 1], bv = c2[kk + 1];
                            y11 = fma(m[kk], av, y11);
                            y21 = fma(d[kk], av, y21);
                            y21 = fma(m[kk], bv, y21);
                        }
                    }
                    ya_[0] = y10;
                    yb_[0] = kFold ? fma(g.alpha, y10, g.beta * y20) : y20;
                    if (ytwo) {
                        ya_[LS] = y11;
                        yb_[LS] = kFold ? fma(g.alpha, y11, g.beta * y21) : y21;
                    }
                }
            }
            __syncthreads();
        }
    } else {
        // ---- x pass: tasks t = tid'' + i TXT (output columns 2i, 2i+1 of tile row r);
        // interior pairs first, padded to whole waves
        const int txd = tid - TZT - TYT;
        const int npx = (TXv + 1) >> 1;
        int ia = X.ilo - x0;
        ia = ia <= 0 ? 0 : (ia + 1) >> 1;
        int ib = X.ihi - x0 - 1;
        ib = ib < 0 ? 0 : (ib >> 1) + 1;
        ia = min(ia, npx);
        ib = min(max(ib, ia), npx);
        const int nI = ib - ia, nB = npx - nI;
        const int nXI = TYv * nI, nXIp = (nXI + 63) & ~63, nXB = TYv * nB;
        int ti[NX], tr[NX];   // column pair xi (flags in the high bits: interior, valid), row
        unsigned tp[NX];      // byte offset of the pair inside an output plane
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            const int t = txd + i * TXT;
            bool xv, xint;
            int xr, xi;
            if (t < nXIp) {
                xint = true;
                xv = t < nXI;
                const int u = xv ? t : 0;
                xr = nI > 0 ? u / nI : 0;
                xi = ia + (u - xr * nI);
            } else {
                xint = false;
                const int t0 = t - nXIp;
                xv = t0 < nXB;
                const int u = xv ? t0 : 0;
                xr = nB > 0 ? u / nB : 0;
                const int j = u - xr * nB;
                xi = j < ia ? j : j + nI;
            }
            xi = min(xi, npx - 1);
            ti[i] = xi | (xint ? 1 << 16 : 0) | (xv ? 1 << 17 : 0);
            tr[i] = xr;
            tp[i] = (unsigned)((y0 + xr) * X.R + x0 + 2 * xi) * 8u;
        }
        const size_t oplane = (size_t)X.R * Y.R;
        for (int k = 0; k < TZv + 2; ++k) {
            const bool live = k >= 2;
            const int oz = max(z0 + k - 2, 0);
            // uniform scalar loads of the plane's scale and source factors
            const double sz = ((cdp)Z.S)[oz], fz = ((cdp)Z.F)[oz];
            const size_t pb = live ? (size_t)oz * oplane : 0;
            const size_t pn = live ? oplane : 0;
            const auto ro = buf(g.out + pb, pn);
            double xim[W], xid[W];
            uniform_row<W>(xim, xid, X.M, X.D, opaque(X.ilo <= X.ihi ? X.ilo : 0));
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                const int xi = ti[i] & 0xffff, xr = tr[i];
                const bool xint = (ti[i] & (1 << 16)) != 0, xv = (ti[i] & (1 << 17)) != 0;
                const bool xtwo = x0 + 2 * xi + 1 < x1;
                const unsigned opair = xv && xtwo ? tp[i] : kOOB, osing = xv && !xtwo ? tp[i] : kOOB;
                const int xrd = xr * LS + 2 * xi;
                const dv2* p1 = reinterpret_cast<const dv2*>(sY + (k & 1) * 2 * ysz + xrd);
                const dv2* p2 = reinterpret_cast<const dv2*>(sY + (k & 1) * 2 * ysz + ysz + xrd);
                double a[2 * P + 2], b[2 * P + 2];
#pragma unroll
                for (int kk = 0; kk < P + 1; ++kk) {
                    const dv2 va = p1[kk], vb = p2[kk];
                    a[2 * kk] = va.x;
                    a[2 * kk + 1] = va.y;
                    b[2 * kk] = vb.x;
                    b[2 * kk + 1] = vb.y;
                }
                double o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0;
                if (!xv || !live) {
                } else if (xint) {
                    xcol<P, kFold>(a, b, 0, xim, xid, o0, o1);
                    xcol<P, kFold>(a, b, 1, xim, xid, o2, o3);
                } else {
                    double m[W], d[W];
                    lds_taps<W>(m, d, tx_ + (2 * xi) * 2 * W);
                    xcol<P, kFold>(a, b, 0, m, d, o0, o1);
                    lds_taps<W>(m, d, tx_ + (2 * xi + 1) * 2 * W);
                    xcol<P, kFold>(a, b, 1, m, d, o2, o3);
                }
                double v0, v1;
                if constexpr (kFold) {
                    v0 = fma(g.beta, o1, o0);
                    v1 = fma(g.beta, o3, o2);
                } else {
                    const auto rm = buf(g.omass + pb, pn);
                    bstore2<kKeep>(rm, opair, o0, o2);
                    bstore<kKeep>(rm, osing, o0);
                    v0 = fma(g.alpha, o0, g.beta * o1);
                    v1 = fma(g.alpha, o2, g.beta * o3);
                }
                // the products in the order of the 2D kernel's epilogue
                dv2 sxv = {1.0, 1.0}, fxv = {1.0, 1.0};
                double syz = 1.0;
                if constexpr ((MODE & kScaleSrc) != 0) {
                    sxv = *reinterpret_cast<const dv2*>(sfx + 2 * xi);
                    fxv = *reinterpret_cast<const dv2*>(sfx + pl.TX + 2 * xi);
                    syz = sfy[xr] * sz;
                    const double fyz = sfy[pl.TY + xr] * fz;
                    v0 = fma(g.gsep, fxv.x * fyz, v0);
                    v1 = fma(g.gsep, fxv.y * fyz, v1);
                }
                if constexpr ((MODE & kFarr) != 0) {
                    const auto rf = buf(g.farr + pb, pn);
                    const dv2 fa = bload2(rf, opair);
                    const double fs = bload(rf, osing);
                    v0 = fma(g.garr, xtwo ? fa.x : fs, v0);
                    v1 = fma(g.garr, fa.y, v1);
                }
                if constexpr ((MODE & kScaleSrc) != 0) {
                    v0 *= sxv.x * syz;
                    v1 *= sxv.y * syz;
                }
                bstore2<kKeep>(ro, opair, v0, v1);
                bstore<kKeep>(ro, osing, v0);
            }
            __syncthreads();
        }
    }
}

template <int P, int MODE>
__global__ __launch_bounds__(kMaxNT3, 4) void apply3d_kernel(ApplyArgs g, Plan3D pl)
{
    apply3d_tile<P, MODE>(g, pl, xcd_logical_block((int)blockIdx.x, pl.nblk));
}

}  // namespace iga
