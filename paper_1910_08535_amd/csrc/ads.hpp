// Alternating-directions direct solve with the Galerkin mass matrix (Section 4.1).
//
// The d-dimensional Galerkin mass is the Kronecker product M_z (x) M_y (x) M_x of the
// 1D matrices M_a(i, j) = int B_i B_j, so its inverse is the product of the 1D inverses:
// the solve is three families of 1D banded systems with many right-hand sides, one
// family per axis, each line independent of the others.  Each M_a is symmetric
// positive definite with bandwidth p; it is factorized once as M_a = L_a L_a^T and
// every solve runs a forward and a backward substitution along every line.
#pragma once
#include "common.hpp"

namespace iga {

// Row r of a factor table holds [L(r, r-P), ..., L(r, r-1), 1 / L(r, r)] (entries of
// columns < 0 are 0), and P rows of zeros follow the last row so that the backward
// substitution needs no bounds test.
template <int P>
constexpr int factor_row() { return P + 1; }

// ---------------------------------------------------------------------------------
// Banded Cholesky factor of one axis (one workgroup).
//   M: band rows of M_a, W = 2P+1 slots per row, slot k <-> column r + k - P.
//   Rows ilo..ihi of M are bitwise identical (the interior element classes).  The
//   recurrence for row r reads only row r of M and the factor rows r-P .. r-1, so once
//   P+1 consecutive factor rows inside the interior are bitwise identical, every later
//   interior row equals them: the workgroup copies that row over the rest of the
//   interior and thread 0 carries on after it.  Without such a repeat the recurrence
//   simply runs to the end.
// ---------------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ void chol_row(const double* __restrict__ m, const double (&win)[P][P + 1],
                                         int r, double (&l)[P + 1])
{
    // l[k] = L(r, j), j = r - P + k; the window holds rows r-P .. r-1 (win[k] is row r-P+k)
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double s = m[k];
#pragma unroll
        for (int t = 0; t < k; ++t) s = fma(-l[t], win[k][t - k + P], s);
        l[k] = r - P + k >= 0 ? s * win[k][P] : 0.0;
    }
    double d = m[P];
#pragma unroll
    for (int t = 0; t < P; ++t) d = fma(-l[t], l[t], d);
    l[P] = 1.0 / sqrt(d);
}

template <int P>
__global__ __launch_bounds__(256) void chol_band_kernel(const double* __restrict__ M, int N, int ilo,
                                                        int ihi, double* __restrict__ L)
{
    constexpr int W = 2 * P + 1, FR = P + 1;
    __shared__ int s_from, s_to;
    __shared__ double s_row[FR];
    double win[P][P + 1];
    int resume = N;
    if (threadIdx.x == 0) {
        s_from = s_to = 0;
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int t = 0; t <= P; ++t) win[k][t] = 0.0;
        for (int r = 0; r < N; ++r) {
            double m[W];
            const int src = (r >= ilo && r <= ihi) ? ilo : r;
#pragma unroll
            for (int k = 0; k < W; ++k) m[k] = M[(size_t)src * W + k];
            double l[P + 1];
            chol_row<P>(m, win, r, l);
#pragma unroll
            for (int k = 0; k <= P; ++k) L[(size_t)r * FR + k] = l[k];
            bool same = r >= ilo && r < ihi;
#pragma unroll
            for (int j = 0; j < P; ++j)
#pragma unroll
                for (int k = 0; k <= P; ++k)
                    same = same && __double_as_longlong(win[j][k]) == __double_as_longlong(l[k]);
#pragma unroll
            for (int j = 0; j + 1 < P; ++j)
#pragma unroll
                for (int k = 0; k <= P; ++k) win[j][k] = win[j + 1][k];
#pragma unroll
            for (int k = 0; k <= P; ++k) win[P - 1][k] = l[k];
            if (same) {   // rows r+1 .. ihi equal row r
                s_from = r + 1;
                s_to = ihi + 1;
#pragma unroll
                for (int k = 0; k <= P; ++k) s_row[k] = l[k];
                resume = ihi + 1;
                break;
            }
        }
    }
    __syncthreads();
    const int from = s_from, to = s_to;
    for (size_t i = (size_t)from * FR + threadIdx.x; i < (size_t)to * FR; i += blockDim.x)
        L[i] = s_row[(i - (size_t)from * FR) % FR];
    // the zero rows after the last row
    for (int i = threadIdx.x; i < P * FR; i += blockDim.x) L[(size_t)N * FR + i] = 0.0;
    if (threadIdx.x == 0) {
        // the window after the copied rows: P copies of the repeated row
        for (int r = resume; r < N; ++r) {
            double m[W];
#pragma unroll
            for (int k = 0; k < W; ++k) m[k] = M[(size_t)r * W + k];
            double l[P + 1];
            chol_row<P>(m, win, r, l);
#pragma unroll
            for (int k = 0; k <= P; ++k) L[(size_t)r * FR + k] = l[k];
#pragma unroll
            for (int j = 0; j + 1 < P; ++j)
#pragma unroll
                for (int k = 0; k <= P; ++k) win[j][k] = win[j + 1][k];
#pragma unroll
            for (int k = 0; k <= P; ++k) win[P - 1][k] = l[k];
        }
    }
}

// ---------------------------------------------------------------------------------
// One family of 1D solves: x = (L L^T)^{-1} b along every line of one axis.
// Line t = (o, i), o in [0, lines / inner), i in [0, inner): element r (0 <= r < n) of
// the line sits at o * n * inner + r * inner + i.  So inner = 1 walks x-lines (rows of
// the array), inner = N_x walks y-lines and inner = N_x N_y walks z-lines; consecutive
// threads take consecutive i, which makes the y and z families' accesses coalesced.
// One thread per line: the forward substitution writes y over x, the backward one
// reads it back in reverse.  Each direction keeps the next U values of its line in
// flight (double-buffered), so that the recurrence waits on memory once per block.
// x may equal b.  L rows are uniform across a wave (scalar loads).
// ---------------------------------------------------------------------------------
constexpr int kAdsBlock = 256;

template <int P>
__global__ __launch_bounds__(kAdsBlock) void ads_sweep_kernel(const double* __restrict__ L, int n,
                                                              long long lines, long long inner,
                                                              const double* b, double* x)
{
    constexpr int FR = P + 1, U = 16;
    const long long t = (long long)blockIdx.x * kAdsBlock + threadIdx.x;
    if (t >= lines) return;
    const long long o = t / inner, i = t - o * inner;
    const double* bl = b + o * (long long)n * inner + i;
    double* xl = x + o * (long long)n * inner + i;

    // forward: y_r = (b_r - sum_k L(r, r-P+k) y_{r-P+k}) / L(r, r)
    double yw[P];
#pragma unroll
    for (int k = 0; k < P; ++k) yw[k] = 0.0;
    double cur[U], nxt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = bl[(long long)min(u, n - 1) * inner];
    for (int r0 = 0; r0 < n; r0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = bl[(long long)min(r0 + U + u, n - 1) * inner];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 + u;
            if (r < n) {
                const double* lr = L + (size_t)r * FR;
                double s = cur[u];
#pragma unroll
                for (int k = 0; k < P; ++k) s = fma(-lr[k], yw[k], s);
                const double y = s * lr[P];
                xl[(long long)r * inner] = y;
#pragma unroll
                for (int k = 0; k + 1 < P; ++k) yw[k] = yw[k + 1];
                yw[P - 1] = y;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }

    // backward: x_r = (y_r - sum_{k=1..P} L(r+k, r) x_{r+k}) / L(r, r); the zero rows
    // after the table make the terms beyond the line vanish
    double xw[P];   // xw[k-1] = x_{r+k}
#pragma unroll
    for (int k = 0; k < P; ++k) xw[k] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = xl[(long long)max(n - 1 - u, 0) * inner];
    for (int r0 = n - 1; r0 >= 0; r0 -= U) {
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = xl[(long long)max(r0 - U - u, 0) * inner];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 - u;
            if (r >= 0) {
                double s = cur[u];
#pragma unroll
                for (int k = P; k >= 1; --k) s = fma(-L[(size_t)(r + k) * FR + P - k], xw[k - 1], s);
                const double v = s * L[(size_t)r * FR + P];
                xl[(long long)r * inner] = v;
#pragma unroll
                for (int k = P - 1; k >= 1; --k) xw[k] = xw[k - 1];
                xw[0] = v;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
}

}  // namespace iga
