// Refined test space (Section 2): more test elements than trial elements.
//
// Each trial element is split into rho equal refined elements, and the test B-splines
// Bhat_m of degree p on the refined open knots are summed in sets: row i takes
// T_i = sum_{m = a_i}^{b_i} Bhat_m, which is 1 on the refined elements [a_i, b_i - p] (the
// row's cell) and ramps over p refined elements on each side (not at the domain's ends).
// The cells partition the axis at the midpoints of consecutive Greville abscissae of the
// trial knots, rounded to refined element boundaries, so cell i sits at the centre of
// supp B_i and the square system [int T_i F(B_j)] is regular.  Its rows are integrated
// with the context's Gauss rule on every refined element.  The factors are banded like
// the other forms (the host checks that every row's columns lie in r-p .. r+p), so every
// kernel that applies PG rows applies these, and the mass factor is factorized (banded
// LU, no pivoting) for the alternating-directions solve.
#pragma once
#include "ads.hpp"
#include "common.hpp"
#include "tables.hpp"

namespace iga {

// G_j = p * (Greville abscissa of B_j) in element units: the sum of knots j+1 .. j+p.
__host__ __device__ inline long long greville_sum(int j, int p, int ne)
{
    long long s = 0;
    for (int k = j + 1; k <= j + p; ++k) {
        const int t = k - p;
        s += t < 0 ? 0 : (t > ne ? ne : t);
    }
    return s;
}

// First refined element of cell i (i = 0 .. N): 0, the rounded midpoints, ne * rho.
__host__ __device__ inline long long refined_cut(int i, int p, int ne, int rho)
{
    const int N = ne + p;
    if (i <= 0) return 0;
    if (i >= N) return (long long)ne * rho;
    const long long g = greville_sum(i - 1, p, ne) + greville_sum(i, p, ne);
    return (rho * g + p) / (2 * p);
}

// Rows of one axis (blockIdx.y = axis of the set, whose rho is rho[axis]): the PG mass
// and Laplacian factors int T_i B_j, int T_i B_j'' (slot k <-> column i + k - p), 1 / int T_i
// and int T_i sin(pi x), one thread per row.
__global__ void refined_tables_kernel(AxisSet set, int3 rho3)
{
    const AxisTables& t = set.t[blockIdx.y];
    const int rho = blockIdx.y == 0 ? rho3.x : (blockIdx.y == 1 ? rho3.y : rho3.z);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= t.N) return;
    const int p = t.p, W = t.W, ne = t.ne;
    const long long ns = (long long)ne * rho;
    const long long a = refined_cut(i, p, ne, rho), b = refined_cut(i + 1, p, ne, rho) - 1 + p;
    const long long klo = a - p > 0 ? a - p : 0, khi = b < ns - 1 ? b : ns - 1;
    const double len_dom = t.hi - t.lo;
    const double inv_h = ne / len_dom, inv_hs = (double)ns / len_dom, h = len_dom / ne;
    const double pi = 3.14159265358979323846;
    double am[2 * kMaxP + 1], ad[2 * kMaxP + 1];
    for (int k = 0; k < W; ++k) am[k] = ad[k] = 0.0;
    double len = 0.0, fsin = 0.0;
    for (long long k = klo; k <= khi; ++k) {
        const int e = (int)(k / rho);
        const int ks = (int)(k - (long long)e * rho);
        for (int q = 0; q < t.nq; ++q) {
            const double s = t.gs[q], w = t.gw[q] / rho;
            double Bh[3][kMaxP + 1];
            basis_ders(p, (int)ns, (int)k, s, inv_hs, Bh);
            double T = 0.0;
            for (int m = 0; m <= p; ++m)
                if (k + m >= a && k + m <= b) T += Bh[0][m];
            if (T == 0.0) continue;
            const double st = (ks + s) / rho;
            double Bt[3][kMaxP + 1];
            basis_ders(p, ne, e, st, inv_h, Bt);
            const double wT = w * T;
            for (int m = 0; m <= p; ++m) {
                const int slot = e + m - i + p;
                if (slot < 0 || slot >= W) continue;   // excluded by the host's band check
                am[slot] = fma(wT, Bt[0][m], am[slot]);
                ad[slot] = fma(wT, Bt[2][m], ad[slot]);
            }
            len += wT;
            fsin = fma(wT, sin(pi * (t.lo + h * (e + st))), fsin);
        }
    }
    for (int k = 0; k < W; ++k) {
        t.pm[(size_t)i * W + k] = am[k];
        t.pd[(size_t)i * W + k] = ad[k];
    }
    t.inv_len[i] = 1.0 / len;
    t.fs_pg[i] = fsin;
}

// Banded LU (no pivoting) of one axis' PG mass factor, one thread: A = L U with L unit
// lower and U upper, both of bandwidth P, into the sweep tables of the solve
// (F[r] = [L(r, r-P), ..., L(r, r-1), 1], B[r] = [U(r, r+1) d_r, ..., U(r, r+P) d_r, d_r],
// d_r = 1 / U(r, r)), and kFactorPad zero rows after each.
template <int P>
__global__ void lu_band_kernel(const double* __restrict__ A, int N, double* __restrict__ F,
                               double* __restrict__ B)
{
    constexpr int FR = P + 1;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    lu_rows<P>(A, 0, N, F, B);
    for (int i = 0; i < kFactorPad * FR; ++i) F[(size_t)N * FR + i] = B[(size_t)N * FR + i] = 0.0;
}

}  // namespace iga
