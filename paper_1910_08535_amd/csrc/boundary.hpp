// Boundary terms of the Laplace problem with mixed conditions (Section 4.3).
//
// Integrating the Laplacian back by parts leaves, on a Neumann side G of the boundary,
// the flux of u_h against the test function; the Neumann datum G enters the right-hand
// side the same way:
//     b_r += alpha int_G T_r du_h/dn dS + beta int_G T_r G dS,
// T_r = B_r (Galerkin) or the indicator of the span S_r (PG).  On a side x_a = const
// the test function factors into its normal part (PG: 1 when the span reaches the side;
// Galerkin: B_{r_a} at the side) and its tangential part, and du_h/dn at the side is
// the trace t_j = n sum_k B'_{j_a}(side) u_{j_a, j} of the p+1 B-splines of the end
// element, so the flux rows are the tangential mass rows applied to t.  Zero Dirichlet
// conditions replace the rows of the B-splines living on a side by identity rows.
#pragma once
#include "common.hpp"
#include "source.hpp"
#include "tables.hpp"

namespace iga {

struct SideArgs {
    int dim, a, hi;           // normal axis, upper (1) or lower (0) end
    int nt;                   // tangential axes (dim - 1)
    int tb[2];                // tangential axes, increasing
    int p, pg;
    int N[3], R[3];           // basis and row counts per axis (1 beyond dim)
    int ne_a;                 // elements along the normal axis
    double inv_h_a;
    const double* M[2];       // tangential mass bands: PG int_{S_r} B_j, Galerkin int B_i B_j
    SrcAxis src[2];           // tangential Gauss rules and basis (for G)
    const int* first_a;       // PG spans of the normal axis
    const int* last_a;
    int rlo, rhi;             // normal rows to examine (inclusive)
    const double* u;
    const double* g;          // G at the side's Gauss points (first tangential axis fastest)
    double g_const, alpha, beta;
    double* b;
};

__device__ __forceinline__ size_t row_index(const int r[3], const int R[3])
{
    return ((size_t)r[2] * R[1] + r[1]) * R[0] + r[0];
}

// One thread per tangential row (r1, r2); in 1D the side is a point and one thread
// does it all.
__global__ void boundary_kernel(SideArgs s)
{
    const int n1 = s.nt > 0 ? s.R[s.tb[0]] : 1;
    const int n2 = s.nt > 1 ? s.R[s.tb[1]] : 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n1 * n2) return;
    const int r1 = idx % n1, r2 = idx / n1;
    const int p = s.p, W = 2 * p + 1;
    // B-splines of the end element and their derivatives at the side
    const int e = s.hi ? s.ne_a - 1 : 0;
    double B[3][kMaxP + 1];
    basis_ders(p, s.ne_a, e, s.hi ? 1.0 : 0.0, s.inv_h_a, B);
    const double nrm = s.hi ? 1.0 : -1.0;

    double val = 0.0;
    if (s.nt == 0) {   // 1D: the side is the end point
        int j[3] = {0, 0, 0};
        double t = 0.0;
        for (int k = 0; k <= p; ++k) {
            j[s.a] = e + k;
            t = fma(B[1][k], s.u ? s.u[row_index(j, s.N)] : 0.0, t);
        }
        val = s.alpha * nrm * t + s.beta * (s.g_const + (s.g ? s.g[0] : 0.0));
    } else if (s.alpha != 0.0) {
        // flux: tangential mass rows applied to the normal-derivative trace
        double flux = 0.0;
        const int k2n = s.nt > 1 ? W : 1;
        for (int k2 = 0; k2 < k2n; ++k2) {
            int c2 = 0;
            double m2 = 1.0;
            if (s.nt > 1) {
                c2 = r2 + k2 - p;
                if (c2 < 0 || c2 >= s.N[s.tb[1]]) continue;
                m2 = s.M[1][(size_t)r2 * W + k2];
                if (m2 == 0.0) continue;
            }
            for (int k1 = 0; k1 < W; ++k1) {
                const int c1 = r1 + k1 - p;
                if (c1 < 0 || c1 >= s.N[s.tb[0]]) continue;
                const double m1 = s.M[0][(size_t)r1 * W + k1];
                if (m1 == 0.0) continue;
                int j[3] = {0, 0, 0};
                j[s.tb[0]] = c1;
                if (s.nt > 1) j[s.tb[1]] = c2;
                double t = 0.0;
                for (int k = 0; k <= p; ++k) {
                    j[s.a] = e + k;
                    t = fma(B[1][k], s.u[row_index(j, s.N)], t);
                }
                flux = fma(m1 * m2, t, flux);
            }
        }
        val = s.alpha * nrm * flux;
    }
    if (s.nt > 0 && s.beta != 0.0) {
        // G: Gauss sums over the tangential test function (span elements or supp B_r)
        const SrcAxis& A1 = s.src[0];
        const SrcAxis& A2 = s.src[1];
        const int e1lo = s.pg ? A1.first[r1] : max(0, r1 - p);
        const int e1hi = s.pg ? A1.last[r1] : min(A1.ne - 1, r1);
        int e2lo = 0, e2hi = 0;
        if (s.nt > 1) {
            e2lo = s.pg ? A2.first[r2] : max(0, r2 - p);
            e2hi = s.pg ? A2.last[r2] : min(A2.ne - 1, r2);
        }
        const size_t ng1 = (size_t)A1.ne * A1.nq;
        double gs = 0.0;
        for (int e2 = e2lo; e2 <= e2hi; ++e2)
            for (int q2 = 0; q2 < (s.nt > 1 ? A2.nq : 1); ++q2) {
                const double w2 = s.nt > 1 ? (s.pg ? A2.gw[q2] : wbasis(A2, e2, q2, r2 - e2)) : 1.0;
                for (int e1 = e1lo; e1 <= e1hi; ++e1)
                    for (int q1 = 0; q1 < A1.nq; ++q1) {
                        const double w1 = s.pg ? A1.gw[q1] : wbasis(A1, e1, q1, r1 - e1);
                        double gv = s.g_const;
                        if (s.g) gv += s.g[((size_t)e2 * A2.nq + q2) * ng1 + (size_t)e1 * A1.nq + q1];
                        gs = fma(w1 * w2, gv, gs);
                    }
            }
        val = fma(s.beta, gs, val);
    }
    // add into every normal row whose test function reaches the side
    int r[3] = {0, 0, 0};
    if (s.nt > 0) r[s.tb[0]] = r1;
    if (s.nt > 1) r[s.tb[1]] = r2;
    for (int ra = s.rlo; ra <= s.rhi; ++ra) {
        double wa;
        if (s.pg) {
            const bool touch = s.hi ? s.last_a[ra] == s.ne_a - 1 : s.first_a[ra] == 0;
            wa = touch ? 1.0 : 0.0;
        } else {
            const int k = ra - e;
            wa = (k >= 0 && k <= p) ? B[0][k] : 0.0;
        }
        if (wa == 0.0) continue;
        r[s.a] = ra;
        const size_t o = row_index(r, s.R);
        s.b[o] = fma(wa, val, s.b[o]);
    }
}

// Identity rows for the B-splines living on one side: rows[r] = u ? u[r] : 0, one thread
// per row of the face (the row index along the normal axis is 0 or N_a - 1).
__global__ void dirichlet_kernel(int a, int hi, int3 N, const double* u, double* rows)
{
    const int n[3] = {N.x, N.y, N.z};
    int tb[2], nt = 0;
    for (int b = 0; b < 3; ++b)
        if (b != a) tb[nt++] = b;
    const int n1 = n[tb[0]], n2 = n[tb[1]];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n1 * n2) return;
    int r[3];
    r[tb[0]] = idx % n1;
    r[tb[1]] = idx / n1;
    r[a] = hi ? n[a] - 1 : 0;
    const size_t o = row_index(r, n);
    rows[o] = u ? u[o] : 0.0;
}

}  // namespace iga
