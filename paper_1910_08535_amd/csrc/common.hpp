// common.hpp -- types shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iga {

constexpr int kMaxP = 3;      // kernels are instantiated for p = 2, 3
constexpr int kMaxNq = 16;    // Gauss points per element per axis
constexpr int kBlock = 256;   // threads per workgroup of the tiled kernels (4 wave64)

// One axis of a tensor-product operator given by banded 1D factors of width
// W = 2p+1: entry k of row r multiplies coefficient r + k - p.
struct AxisOp {
    const double* M;   // [R][W] mass-type factor
    const double* D;   // [R][W] operator factor
    const double* S;   // [R] output scale (inverse span length of the lumped step) or null
    const double* F;   // [R] separable source factor or null
    int R;             // rows
    int N;             // basis functions (columns)
    // Rows ilo..ihi (empty when ilo > ihi) have bitwise identical entries in M and D:
    // rows whose elements and B-splines all lie away from the repeated end knots (the
    // tables evaluate B-splines in element-local knot units, so every such element
    // yields the same values, summed in the same order).
    int ilo, ihi;
};

// out_r  = S(r) * ( alpha (Mass u)_r + beta (Lap u)_r + gsep * prod_a F_a(r_a) + garr * farr_r )
// omass_r = (Mass u)_r            (written when omass != null)
// with Mass = prod_a M_a and Lap = sum_t prod_a (a == t ? D_a : M_a) (Kronecker, x fastest).
struct ApplyArgs {
    AxisOp ax[3];
    const double* u;      // (N_z, N_y, N_x)
    double* out;          // (R_z, R_y, R_x) or null
    double* omass;        // (R_z, R_y, R_x) or null
    const double* farr;   // (R_z, R_y, R_x) or null
    double alpha, beta, gsep, garr;
};

// Launch geometry of the tiled kernels: output tiles of TX x TY (x TZ planes in 3D),
// enumerated x fastest, then y, then z-chunk.
struct TileGrid {
    int tx, ty, tz;       // tiles along each axis
    int TZ;               // planes per z-chunk (3D)
    int nblk;             // tx * ty * tz
};

// XCD-aware block order: gfx950 dispatches consecutive workgroups round-robin over its
// 8 XCDs, each with a private L2.  Give every XCD a contiguous run of logical tiles so
// that neighbouring tiles (which share p-wide halos) mostly land in the same L2.
__device__ __forceinline__ int xcd_logical_block(int bid, int nblk)
{
    const int q = nblk >> 3, r = nblk & 7;
    const int x = bid & 7, k = bid >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Elements of an axis fall into at most 2p+1 classes by their local knot pattern: the
// first p elements, the interior (all alike), the last p.  Basis values at the Gauss
// points depend only on the class, so they are evaluated once per class.
__host__ __device__ inline int n_classes(int p, int ne)
{
    return ne <= 2 * p + 1 ? ne : 2 * p + 1;
}

__host__ __device__ inline int class_of(int e, int p, int ne)
{
    if (ne <= 2 * p + 1) return e;
    return e < p ? e : (e > ne - 1 - p ? e - (ne - (2 * p + 1)) : p);
}

__host__ __device__ inline int class_element(int c, int p, int ne)
{
    if (ne <= 2 * p + 1) return c;
    return c <= p ? c : ne - (2 * p + 1) + c;
}

}  // namespace iga
