// tables.hpp -- set-up kernels: per-axis Gauss rule, B-spline values at the Gauss
// points, and the banded 1D factors of the Galerkin and Petrov-Galerkin matrices.
//
// Everything here runs once per context, so the kernels favour clarity over speed.
// The hot kernels (apply.hpp) only read the tables built here.
#pragma once

#include "common.hpp"

namespace iga {

// Legendre polynomial P_n(z) and its derivative, by the three-term recurrence.
__device__ __forceinline__ void legendre(int n, double z, double* pn, double* dpn)
{
    double pm1 = 1.0, p0 = z;
    if (n == 0) { *pn = 1.0; *dpn = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        const double p1 = ((2.0 * k - 1.0) * z * p0 - (k - 1.0) * pm1) / (double)k;
        pm1 = p0;
        p0 = p1;
    }
    *pn = p0;
    *dpn = (double)n * (z * p0 - pm1) / (z * z - 1.0);
}

// Node i (ascending) and weight of the n-point Gauss-Legendre rule on [-1, 1]:
// Newton's method from Tricomi's asymptotic estimate of the (n-i)-th largest root.
__device__ void gauss_node(int n, int i, double* x, double* w)
{
    const int k = n - i;
    const double nn = (double)n;
    double z = (1.0 - 1.0 / (8.0 * nn * nn) + 1.0 / (8.0 * nn * nn * nn)) *
               cos(M_PI * (4.0 * k - 1.0) / (4.0 * nn + 2.0));
    // quadratic convergence: once a step is below 1e-15 the iterate is exact to rounding
    double pn, dp;
    for (int it = 0; it < 30; ++it) {
        legendre(n, z, &pn, &dp);
        const double dz = pn / dp;
        z -= dz;
        if (fabs(dz) <= 1e-15) break;
    }
    legendre(n, z, &pn, &dp);
    *x = z;
    *w = 2.0 / ((1.0 - z * z) * dp * dp);
}

// Values, first and second derivatives of the p+1 B-splines e..e+p that can be nonzero
// on element e, at the point with local coordinate s in [0, 1] of that element: bottom-up
// triangle of the Cox-de Boor recurrence for degrees 0..p, then the derivative relation
//   d/dx B_{j,k} = k ( B_{j,k-1}/(t_{j+k}-t_j) - B_{j+1,k-1}/(t_{j+k+1}-t_{j+1}) )
// applied once (first derivatives of degrees p-1 and p) and twice (second, degree p).
// The recurrence runs in element units relative to element e: knot t_k becomes the small
// integer clamp(k-p, 0, ne) - e, so every difference is exact however fine the mesh, and
// the derivatives are scaled by 1/h and 1/h^2 at the end (uniform elements of length h).
// out[m][a] = m-th derivative of B_{e+a}.
__device__ __forceinline__ double local_knot(int k, int p, int ne, int e)
{
    const int i = k - p < 0 ? 0 : (k - p > ne ? ne : k - p);
    return (double)(i - e);
}

__device__ void basis_ders(int p, int ne, int e, double s, double inv_h,
                           double out[3][kMaxP + 1])
{
    const int mu = e + p;   // knot interval [t_mu, t_{mu+1})
    // V[k][i] = B_{mu-k+i, k}(s), i = 0..k
    double V[kMaxP + 1][kMaxP + 1];
    V[0][0] = 1.0;
    for (int k = 1; k <= p; ++k) {
        for (int i = 0; i <= k; ++i) {
            const int j = mu - k + i;
            const double tj = local_knot(j, p, ne, e);
            const double tjk = local_knot(j + k, p, ne, e);
            const double tj1 = local_knot(j + 1, p, ne, e);
            const double tjk1 = local_knot(j + k + 1, p, ne, e);
            const double lft = (i > 0) ? V[k - 1][i - 1] : 0.0;   // B_{j,k-1}
            const double rgt = (i < k) ? V[k - 1][i] : 0.0;       // B_{j+1,k-1}
            double v = 0.0;
            if (tjk > tj) v += (s - tj) / (tjk - tj) * lft;
            if (tjk1 > tj1) v += (tjk1 - s) / (tjk1 - tj1) * rgt;
            V[k][i] = v;
        }
    }
    // first derivatives (per unit of s) of degree k in {p-1, p}: D1[k][i] for B_{mu-k+i, k}
    double D1[kMaxP + 1][kMaxP + 1];
    for (int k = (p >= 2 ? p - 1 : 1); k <= p; ++k) {
        for (int i = 0; i <= k; ++i) {
            const int j = mu - k + i;
            const double tj = local_knot(j, p, ne, e);
            const double tjk = local_knot(j + k, p, ne, e);
            const double tj1 = local_knot(j + 1, p, ne, e);
            const double tjk1 = local_knot(j + k + 1, p, ne, e);
            const double lft = (i > 0) ? V[k - 1][i - 1] : 0.0;
            const double rgt = (i < k) ? V[k - 1][i] : 0.0;
            double d = 0.0;
            if (tjk > tj) d += (double)k / (tjk - tj) * lft;
            if (tjk1 > tj1) d -= (double)k / (tjk1 - tj1) * rgt;
            D1[k][i] = d;
        }
    }
    for (int i = 0; i <= p; ++i) {
        out[0][i] = V[p][i];
        out[1][i] = D1[p][i] * inv_h;
        double d2 = 0.0;
        if (p >= 2) {
            const int j = mu - p + i;
            const double tj = local_knot(j, p, ne, e);
            const double tjk = local_knot(j + p, p, ne, e);
            const double tj1 = local_knot(j + 1, p, ne, e);
            const double tjk1 = local_knot(j + p + 1, p, ne, e);
            const double lft = (i > 0) ? D1[p - 1][i - 1] : 0.0;
            const double rgt = (i < p) ? D1[p - 1][i] : 0.0;
            if (tjk > tj) d2 += (double)p / (tjk - tj) * lft;
            if (tjk1 > tj1) d2 -= (double)p / (tjk1 - tj1) * rgt;
        }
        out[2][i] = d2 * inv_h * inv_h;
    }
}

// Element length and its inverse as every table of an axis forms them.
__host__ __device__ inline double elem_len(double lo, double hi, int ne) { return (hi - lo) / (double)ne; }
__host__ __device__ inline double elem_inv_len(double lo, double hi, int ne) { return (double)ne / (hi - lo); }

// Element sum of W sin(pi x) over the Gauss points of element e: gw[q] = weight x Jacobian,
// gs[q] = local coordinate of point q.
__device__ __forceinline__ double elem_sine_sum(double lo, double hi, int ne, int e, int nq, const double* gw,
                                                const double* gs)
{
    double es = 0.0;
    for (int q = 0; q < nq; ++q) {
        const double x = lo + (hi - lo) * (((double)e + gs[q]) / (double)ne);
        es = fma(gw[q], sin(M_PI * x), es);
    }
    return es;
}

// Support span of PG row r (elements s .. l) and the row's scale 1/|S_r| of the lumped step.
__host__ __device__ inline void support_span(int r, int p, int ne, int* s, int* l)
{
    *s = r - p > 0 ? r - p : 0;
    *l = r < ne - 1 ? r : ne - 1;
}

__host__ __device__ inline double span_scale(int s, int l, int ne, double lo, double hi)
{
    return (double)ne / ((double)(l - s + 1) * (hi - lo));
}

// ---------------------------------------------------------------------------------
// Petrov-Galerkin rows in element units.  With support spans on a uniform axis of at
// least 3p+1 elements, the Gauss sums of a PG row depend on the row only through its
// distance to the nearer end (the B-splines are evaluated in element-local knot units):
// the first 2p rows, the last 2p rows and one interior row are all the distinct rows,
// 4p+1 of them.  Summed with weights w_q / 2 and derivatives per unit of the local
// coordinate they hold for every such axis, and the axis' own rows follow as
//   M_r = h * Mgen_c(r),   D_r = (1/h) * Dgen_c(r),   h = (hi - lo) / ne.
// Layout of one (p, nq) table: Mgen[(4p+1) W] | Dgen[(4p+1) W] | w[nq] | s[nq]
// (Gauss weights on [-1, 1] and the points as local coordinates in [0, 1]).
// ---------------------------------------------------------------------------------
__host__ __device__ inline int pg_generic_min_ne(int p) { return 3 * p + 1; }

__host__ __device__ inline size_t pg_generic_doubles(int p, int nq)
{
    return 2 * (size_t)(4 * p + 1) * (2 * p + 1) + 2 * (size_t)nq;
}

// The distinct row (0 .. 4p) that row r of an axis of R rows equals.
__host__ __device__ inline int pg_row_class(int r, int R, int p)
{
    return r < 2 * p ? r : (r >= R - 2 * p ? 4 * p - (R - 1 - r) : 2 * p);
}

// Taps k of PG row r of an axis: M = h Mgen, D = (1/h) Dgen.
__device__ __forceinline__ void pg_generic_row(const double* gen, int p, int r, int R, double h, double ih,
                                               double* m, double* d)
{
    const int W = 2 * p + 1, c = pg_row_class(r, R, p);
    const double* gm = gen + (size_t)c * W;
    const double* gd = gen + (size_t)(4 * p + 1) * W + (size_t)c * W;
    for (int k = 0; k < W; ++k) {
        m[k] = h * gm[k];
        d[k] = ih * gd[k];
    }
}

// Per-axis device tables.  Layout of one axis (all doubles unless noted):
//   cls[ncls*nq*3*(p+1)]      cls[((c*nq+q)*3 + m)*(p+1) + a] = B^{(m)}_{e+a} at point q of
//                             an element e of class c
//   gw[nq], gs[nq]            weight*Jacobian and local coordinate in [0, 1] of point q
//                             (the same on every element: uniform elements)
//   es[ne], eg[ne*(p+1)]      element sums of W sin(pi x) and of W B_{e+a} sin(pi x)
//   pm[R*W], pd[R*W]          PG factors  int_{S_r} B_j,  int_{S_r} B_j''   (column r+k-p)
//   inv_len[R], fs_pg[R]      1/|S_r|,  int_{S_r} sin(pi x)  (Gauss rule)
//   gm[N*W], gl[N*W], gb[N*W] Galerkin int B_i B_j, int B_i B_j'', -int B_i' B_j'
//   fs_g[N]                   int B_i sin(pi x)  (Gauss rule)
//   first[R], last[R] (int)   PG spans
// pgen points at the element-unit PG rows of (p, nq) (below) when the axis' PG factors are
// taken from them, else it is null.
struct AxisTables {
    int p, ne, nq, N, R, W;
    double lo, hi;
    double *cls, *gw, *gs;
    double *es, *eg;
    double *pm, *pd, *inv_len, *fs_pg;
    double *gm, *gl, *gb, *fs_g;
    int *first, *last;
    const double* pgen;
};

// The tables of every axis of a context, filled by three launches in all.
struct AxisSet {
    AxisTables t[3];
    int dim;
    int kind;         // span kind (iga_spans)
    double* consts;   // {1, 0 x 7} | two int zeros | ones[nones]
    size_t nones;
};

// One workgroup per axis, one thread per (class, Gauss point): the Gauss rule and the
// basis values of the class.
__global__ void class_tables_kernel(AxisSet set)
{
    const AxisTables& t = set.t[blockIdx.x];
    const int idx = threadIdx.x;
    const int nc = n_classes(t.p, t.ne);
    if (idx >= nc * t.nq) return;
    const int c = idx / t.nq, q = idx - c * t.nq;
    double xi, w;
    gauss_node(t.nq, q, &xi, &w);
    // uniform elements: h itself, not a difference of two rounded knots
    const double h = (t.hi - t.lo) / (double)t.ne;
    const double sl = 0.5 * (xi + 1.0);   // local coordinate in [0, 1]
    if (c == 0) {
        t.gw[q] = 0.5 * w * h;
        t.gs[q] = sl;
    }
    double B[3][kMaxP + 1];
    basis_ders(t.p, t.ne, class_element(c, t.p, t.ne), sl, (double)t.ne / (t.hi - t.lo), B);
    for (int m = 0; m < 3; ++m)
        for (int a = 0; a <= t.p; ++a) t.cls[((size_t)idx * 3 + m) * (t.p + 1) + a] = B[m][a];
}

// One thread per element (blockIdx.y = axis): the element sums of the sine source over
// its Gauss points (basis values from the class tables).  Row blockIdx.y == dim fills
// the context's constants when the set carries them.
__global__ void element_tables_kernel(AxisSet set)
{
    if ((int)blockIdx.y == set.dim) {
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 9 + set.nones;
             i += (size_t)gridDim.x * blockDim.x) {
            if (i < 8)
                set.consts[i] = i == 0 ? 1.0 : 0.0;
            else if (i == 8)
                ((int*)(set.consts + 8))[0] = ((int*)(set.consts + 8))[1] = 0;
            else
                set.consts[i] = 1.0;
        }
        return;
    }
    const AxisTables& t = set.t[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= t.ne) return;
    const int np1 = t.p + 1, nb = 3 * np1;
    const int c = class_of(e, t.p, t.ne);
    double eg[kMaxP + 1] = {};
    for (int q = 0; q < t.nq; ++q) {
        const double x = t.lo + (t.hi - t.lo) * (((double)e + t.gs[q]) / (double)t.ne);
        const double sx = sin(M_PI * x), w = t.gw[q];
        const double* B = t.cls + ((size_t)c * t.nq + q) * nb;
        for (int a = 0; a <= t.p; ++a) eg[a] += w * B[a] * sx;
    }
    t.es[e] = elem_sine_sum(t.lo, t.hi, t.ne, e, t.nq, t.gw, t.gs);
    for (int a = 0; a <= t.p; ++a) t.eg[(size_t)e * np1 + a] = eg[a];
}

// One thread per row: the Gauss sums of the banded factors, from the class tables staged
// in LDS.  PG rows never multiply by a test function -- the integrand is summed with
// weight 1 over the span's elements.  Spans of the built-in kinds (kind 0 support, 1
// element) are generated here; caller spans (kind 2) are already in first/last.
__global__ void band_tables_kernel(AxisSet set)
{
    const AxisTables& t = set.t[blockIdx.y];
    const int kind = set.kind;
    extern __shared__ double sb[];
    const int p = t.p, np1 = t.p + 1, nq = t.nq, W = t.W;
    const int nb = 3 * np1, nc = n_classes(p, t.ne);
    double* scls = sb;                       // [nc*nq*3*np1]
    double* sgw = sb + (size_t)nc * nq * nb; // [nq]
    for (int i = threadIdx.x; i < nc * nq * nb; i += blockDim.x) scls[i] = t.cls[i];
    for (int i = threadIdx.x; i < nq; i += blockDim.x) sgw[i] = t.gw[i];
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < t.R) {
        int s, l;
        if (kind == 0) {
            support_span(r, p, t.ne, &s, &l);
            t.first[r] = s;
            t.last[r] = l;
        } else if (kind == 1) {
            s = l = r;
            t.first[r] = s;
            t.last[r] = l;
        } else {
            s = t.first[r];
            l = t.last[r];
        }
        if (t.pgen) {   // support spans, at least 3p+1 elements: scaled element-unit rows
            double m[2 * kMaxP + 1], d[2 * kMaxP + 1];
            pg_generic_row(t.pgen, p, r, t.R, elem_len(t.lo, t.hi, t.ne), elem_inv_len(t.lo, t.hi, t.ne), m, d);
            for (int k = 0; k < W; ++k) {
                t.pm[(size_t)r * W + k] = m[k];
                t.pd[(size_t)r * W + k] = d[k];
            }
        } else {
            for (int k = 0; k < W; ++k) {
                const int j = r + k - p;
                double m0 = 0.0, d0 = 0.0;
                for (int e = s; e <= l; ++e) {
                    const int a = j - e;
                    if (a < 0 || a > p) continue;
                    const double* B = scls + (size_t)class_of(e, p, t.ne) * nq * nb;
                    for (int q = 0; q < nq; ++q) {
                        m0 += sgw[q] * B[q * nb + a];
                        d0 += sgw[q] * B[q * nb + 2 * np1 + a];
                    }
                }
                t.pm[(size_t)r * W + k] = m0;
                t.pd[(size_t)r * W + k] = d0;
            }
        }
        double fs = 0.0;
        for (int e = s; e <= l; ++e) fs += t.es[e];
        t.fs_pg[r] = fs;
        t.inv_len[r] = span_scale(s, l, t.ne, t.lo, t.hi);
    }
    if (r < t.N) {
        const int e0 = r - p < 0 ? 0 : r - p;
        const int e1 = r < t.ne - 1 ? r : t.ne - 1;
        for (int k = 0; k < W; ++k) {
            const int j = r + k - p;
            double gm = 0.0, gl = 0.0, gb = 0.0;
            for (int e = e0; e <= e1; ++e) {
                const int c = r - e, a = j - e;
                if (a < 0 || a > p) continue;
                const double* Bc = scls + (size_t)class_of(e, p, t.ne) * nq * nb;
                for (int q = 0; q < nq; ++q) {
                    const double* B = Bc + q * nb;
                    gm += sgw[q] * B[c] * B[a];
                    gl += sgw[q] * B[c] * B[2 * np1 + a];
                    gb -= sgw[q] * B[np1 + c] * B[np1 + a];
                }
            }
            t.gm[(size_t)r * W + k] = gm;
            t.gl[(size_t)r * W + k] = gl;
            t.gb[(size_t)r * W + k] = gb;
        }
        double fs = 0.0;
        for (int e = e0; e <= e1; ++e) fs += t.eg[(size_t)e * np1 + (r - e)];
        t.fs_g[r] = fs;
    }
}

// The 4p+1 distinct element-unit PG rows of (p, nq), computed on the axis of 3p+1
// elements, where each occurs once (row 2p is its only interior row): one workgroup, one
// thread per (row, tap).  Every sum runs over the row's span elements, then the Gauss
// points, in the order of the per-axis kernel above.
__global__ void pg_generic_kernel(double* gen, int p, int nq)
{
    __shared__ double sw[kMaxNq], ss[kMaxNq];
    __shared__ double scls[(2 * kMaxP + 1) * kMaxNq * 3 * (kMaxP + 1)];
    const int np1 = p + 1, nb = 3 * np1, W = 2 * p + 1;
    const int ne = pg_generic_min_ne(p), nc = n_classes(p, ne);
    const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
    for (int q = tid; q < nq; q += nt) {
        double xi, w;
        gauss_node(nq, q, &xi, &w);
        sw[q] = w;
        ss[q] = 0.5 * (xi + 1.0);
    }
    __syncthreads();
    for (int i = tid; i < nc * nq; i += nt) {
        const int c = i / nq, q = i - c * nq;
        double B[3][kMaxP + 1];
        basis_ders(p, ne, class_element(c, p, ne), ss[q], 1.0, B);
        for (int m = 0; m < 3; ++m)
            for (int a = 0; a <= p; ++a) scls[((size_t)i * 3 + m) * np1 + a] = B[m][a];
    }
    __syncthreads();
    for (int i = tid; i < (4 * p + 1) * W; i += nt) {
        const int rc = i / W, k = i - rc * W;
        const int r = rc;   // R = 4p+1 rows: row rc is distinct row rc
        int s, l;
        support_span(r, p, ne, &s, &l);
        const int j = r + k - p;
        double m0 = 0.0, d0 = 0.0;
        for (int e = s; e <= l; ++e) {
            const int a = j - e;
            if (a < 0 || a > p) continue;
            const double* B = scls + (size_t)class_of(e, p, ne) * nq * nb;
            for (int q = 0; q < nq; ++q) {
                const double w = 0.5 * sw[q];
                m0 += w * B[q * nb + a];
                d0 += w * B[q * nb + 2 * np1 + a];
            }
        }
        gen[i] = m0;
        gen[(size_t)(4 * p + 1) * W + i] = d0;
    }
    for (int q = tid; q < nq; q += nt) {
        gen[2 * (size_t)(4 * p + 1) * W + q] = sw[q];
        gen[2 * (size_t)(4 * p + 1) * W + nq + q] = ss[q];
    }
}

}  // namespace iga
