/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Direct loops over elements, Gauss points and local basis products, with no sum
 * factorization, no blocking and no reordering beyond the definitions:
 *
 *  - B-splines: the Cox-de Boor recursion on the open uniform knot vector of
 *    Section 2 (N = N_e + p functions, p+1 of them nonzero on every element), in
 *    physical coordinates, with derivatives from the derivative recursion.
 *  - Quadrature: Gauss-Legendre (Section 2, Section 4.1), mapped per element,
 *    weight times Jacobian W = w * h / 2.
 *  - Galerkin rows: test with B_i, either integrated by parts
 *    (-int grad B_i . grad u_h) or in the Laplacian form (int B_i Lap u_h),
 *    Section 1.
 *  - Petrov-Galerkin rows: the test function of row r is the indicator of the
 *    span S_r, so the integrand is never multiplied by a test B-spline
 *    (Section 2 "black terms", Section 3, and the piece-wise-constant generation
 *    loops of Section 4.1 and Section 4.3).  The integral over a span is the sum
 *    of the integrals over its elements.
 *  - Explicit dynamics: forward Euler of Section 4.2,
 *    (I_r, u_{t+1}) = (I_r, u_t + dt Lap u_t + dt f), with the left-hand side
 *    lumped by its row sums, sum_j int_{S_r} B_j = |S_r| (partition of unity).
 *
 * Axes beyond dim are carried as one degenerate element with one point of
 * weight 1 and one "basis function" equal to 1 with zero derivatives, so that
 * the three-dimensional loops reduce exactly to the lower-dimensional sums.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;

static const ld PI_L = 3.141592653589793238462643383279502884L;

/* ------------------------------------------------------------------------ */
/* Section 2: open uniform knot vector t_0 .. t_{ne+2p}                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int p;
    long ne;
    ld lo, hi;
} knots_t;

static ld knot(const knots_t *kv, long k)
{
    if (k <= kv->p) return kv->lo;
    if (k >= kv->ne + kv->p) return kv->hi;
    return kv->lo + (kv->hi - kv->lo) * (ld)(k - kv->p) / (ld)kv->ne;
}

/* m-th derivative of B_{j,k} at x, where x lies in the knot interval
   [t_mu, t_{mu+1}).  Cox-de Boor:
     B_{j,0} = 1 on [t_j, t_{j+1}), else 0;
     B_{j,k} = (x - t_j)/(t_{j+k} - t_j) B_{j,k-1}
             + (t_{j+k+1} - x)/(t_{j+k+1} - t_{j+1}) B_{j+1,k-1};
   derivative:
     B^{(m)}_{j,k} = k [ B^{(m-1)}_{j,k-1}/(t_{j+k} - t_j)
                       - B^{(m-1)}_{j+1,k-1}/(t_{j+k+1} - t_{j+1}) ];
   a quotient with a zero denominator is taken as 0. */
static ld bspline(const knots_t *kv, long j, int k, int m, ld x, long mu)
{
    if (m > k) return 0.0L;
    if (k == 0) return (j == mu) ? 1.0L : 0.0L;
    ld tj = knot(kv, j), tjk = knot(kv, j + k);
    ld tj1 = knot(kv, j + 1), tjk1 = knot(kv, j + k + 1);
    ld d1 = tjk - tj, d2 = tjk1 - tj1;
    ld r = 0.0L;
    if (m == 0) {
        if (d1 > 0) r += (x - tj) / d1 * bspline(kv, j, k - 1, 0, x, mu);
        if (d2 > 0) r += (tjk1 - x) / d2 * bspline(kv, j + 1, k - 1, 0, x, mu);
    } else {
        if (d1 > 0) r += (ld)k / d1 * bspline(kv, j, k - 1, m - 1, x, mu);
        if (d2 > 0) r -= (ld)k / d2 * bspline(kv, j + 1, k - 1, m - 1, x, mu);
    }
    return r;
}

/* knot interval index mu with t_mu <= x < t_{mu+1}; the last interval is closed.
   Returns -1 outside [lo, hi]. */
static long find_interval(const knots_t *kv, ld x)
{
    if (x < kv->lo || x > kv->hi) return -1;
    long e = (long)floorl((x - kv->lo) / (kv->hi - kv->lo) * (ld)kv->ne);
    if (e < 0) e = 0;
    if (e > kv->ne - 1) e = kv->ne - 1;
    while (e > 0 && x < knot(kv, e + kv->p)) e--;
    while (e < kv->ne - 1 && x >= knot(kv, e + kv->p + 1)) e++;
    return e + kv->p;
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre quadrature: Newton's method on P_n, evaluated by the        */
/* three-term recurrence k P_k = (2k-1) z P_{k-1} - (k-1) P_{k-2}.            */
/* ------------------------------------------------------------------------ */

static int gauss_legendre_ld(int n, ld *xi, ld *w)
{
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; ++i) {
        ld z = cosl(PI_L * ((ld)i + 0.75L) / ((ld)n + 0.5L));
        ld pn = 0, pnm1 = 0, dp = 1;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((ld)(2 * k - 1) * z * p1 - (ld)(k - 1) * p0) / (ld)k;
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 1) ? z : p1;
            pnm1 = (n == 1) ? 1.0L : p0;
            dp = (ld)n * (z * pn - pnm1) / (z * z - 1.0L);
            ld dz = pn / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        /* recompute P_n' at the converged root */
        {
            ld p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                ld p2 = ((ld)(2 * k - 1) * z * p1 - (ld)(k - 1) * p0) / (ld)k;
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 1) ? z : p1;
            pnm1 = (n == 1) ? 1.0L : p0;
            dp = (ld)n * (z * pn - pnm1) / (z * z - 1.0L);
        }
        /* roots come out descending; store ascending */
        xi[n - 1 - i] = z;
        w[n - 1 - i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
    return 0;
}

int or_gauss_legendre(int nq, double *xi, double *w)
{
    ld x[64], ww[64];
    if (gauss_legendre_ld(nq, x, ww)) return -1;
    for (int i = 0; i < nq; ++i) {
        xi[i] = (double)x[i];
        w[i] = (double)ww[i];
    }
    return 0;
}

int or_basis_eval(int p, long ne, double lo, double hi, double x, int nder, double *out)
{
    if (p < 0 || p > OR_MAXP || ne < 1 || !(lo < hi) || nder < 0 || nder > 2) return -1;
    knots_t kv = {p, ne, lo, hi};
    long N = ne + p;
    for (long i = 0; i < (long)(nder + 1) * N; ++i) out[i] = 0.0;
    long mu = find_interval(&kv, (ld)x);
    if (mu < 0) return 0;
    for (int d = 0; d <= nder; ++d)
        for (long j = 0; j < N; ++j)
            out[d * N + j] = (double)bspline(&kv, j, p, d, (ld)x, mu);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-axis Gauss data: for element e and point q, the physical point, the    */
/* weight times Jacobian, and the values/derivatives of the p+1 B-splines     */
/* e .. e+p that can be nonzero there.                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int p;          /* degree (0 for a degenerate axis) */
    long ne, nb;    /* elements, basis functions */
    int nq;
    ld *x;          /* [ne*nq] */
    ld *W;          /* [ne*nq] */
    ld *B;          /* [(ne*nq)*3*(p+1)]: B[(eq*3 + m)*(p+1) + a] */
    ld *elen;       /* [ne] knot length of element e */
    int real;       /* 0 for an axis beyond dim */
} axis_t;

static void axis_free(axis_t *ax)
{
    free(ax->x);
    free(ax->W);
    free(ax->B);
    free(ax->elen);
}

static int axis_build(axis_t *ax, int p, long ne, double lo, double hi, int nq)
{
    memset(ax, 0, sizeof(*ax));
    ax->p = p;
    ax->ne = ne;
    ax->nb = ne + p;
    ax->nq = nq;
    ax->real = 1;
    ax->x = malloc(sizeof(ld) * ne * nq);
    ax->W = malloc(sizeof(ld) * ne * nq);
    ax->B = malloc(sizeof(ld) * ne * nq * 3 * (p + 1));
    ax->elen = malloc(sizeof(ld) * ne);
    if (!ax->x || !ax->W || !ax->B || !ax->elen) return -1;
    ld xi[64], w[64];
    if (gauss_legendre_ld(nq, xi, w)) return -1;
    knots_t kv = {p, ne, lo, hi};
    for (long e = 0; e < ne; ++e) {
        ld a0 = knot(&kv, e + p), a1 = knot(&kv, e + p + 1);
        ax->elen[e] = a1 - a0;
        for (int q = 0; q < nq; ++q) {
            long eq = e * nq + q;
            ld xx = a0 + (xi[q] + 1.0L) * 0.5L * (a1 - a0);
            ax->x[eq] = xx;
            ax->W[eq] = w[q] * 0.5L * (a1 - a0);
            for (int m = 0; m < 3; ++m)
                for (int a = 0; a <= p; ++a)
                    ax->B[(eq * 3 + m) * (p + 1) + a] = bspline(&kv, e + a, p, m, xx, e + p);
        }
    }
    return 0;
}

/* one element, one point, one function equal to 1 */
static int axis_degenerate(axis_t *ax)
{
    memset(ax, 0, sizeof(*ax));
    ax->p = 0;
    ax->ne = 1;
    ax->nb = 1;
    ax->nq = 1;
    ax->real = 0;
    ax->x = calloc(1, sizeof(ld));
    ax->W = malloc(sizeof(ld));
    ax->B = calloc(3, sizeof(ld));
    ax->elen = malloc(sizeof(ld));
    if (!ax->x || !ax->W || !ax->B || !ax->elen) return -1;
    ax->W[0] = 1.0L;
    ax->B[0] = 1.0L;
    ax->elen[0] = 1.0L;
    return 0;
}

static int check_problem(const or_problem *pb, int need_spans)
{
    if (!pb || pb->dim < 1 || pb->dim > 3 || pb->p < 1 || pb->p > OR_MAXP) return -1;
    for (int a = 0; a < pb->dim; ++a) {
        if (pb->ne[a] < 1 || !(pb->lo[a] < pb->hi[a]) || pb->nq[a] < 1 || pb->nq[a] > 64)
            return -1;
        if (need_spans) {
            if (pb->nspan[a] < 1 || !pb->span_first[a] || !pb->span_last[a]) return -1;
            for (long r = 0; r < pb->nspan[a]; ++r) {
                long s = pb->span_first[a][r], t = pb->span_last[a][r];
                if (s < 0 || t < s || t >= pb->ne[a]) return -1;
            }
        }
    }
    return 0;
}

static int build_axes(const or_problem *pb, axis_t ax[3])
{
    int rc = 0;
    for (int a = 0; a < 3; ++a) {
        if (a < pb->dim)
            rc |= axis_build(&ax[a], pb->p, pb->ne[a], pb->lo[a], pb->hi[a], pb->nq[a]);
        else
            rc |= axis_degenerate(&ax[a]);
    }
    return rc;
}

/* span of row r along axis a (the whole single element on a degenerate axis) */
static void span_of(const or_problem *pb, int a, long r, long *s, long *t)
{
    if (a < pb->dim) {
        *s = pb->span_first[a][r];
        *t = pb->span_last[a][r];
    } else {
        *s = 0;
        *t = 0;
    }
}

/* the source f at the Gauss point with per-axis indices (e[a], q[a]) */
static ld source_at(const or_problem *pb, const axis_t ax[3], const or_source *src,
                    const long e[3], const int q[3])
{
    if (!src) return 0.0L;
    ld f = 0.0L;
    if (src->sin_amp != 0.0) {
        ld s = (ld)src->sin_amp;
        for (int a = 0; a < pb->dim; ++a) s *= sinl(PI_L * ax[a].x[e[a] * ax[a].nq + q[a]]);
        f += s;
    }
    if (src->table) {
        long g[3], ng[3];
        for (int a = 0; a < 3; ++a) {
            g[a] = e[a] * ax[a].nq + q[a];
            ng[a] = ax[a].ne * ax[a].nq;
        }
        f += (ld)src->table[(g[2] * ng[1] + g[1]) * ng[0] + g[0]];
    }
    return f;
}

/* u_h, its gradient and its Laplacian at one Gauss point of element e:
   u_h = sum over the (p+1)^dim local functions of u_j * prod_a B_{j_a}. */
static void trial_at(const axis_t ax[3], const double *u, const long e[3], const int q[3],
                     ld *val, ld grad[3], ld *lap)
{
    *val = 0.0L;
    *lap = 0.0L;
    grad[0] = grad[1] = grad[2] = 0.0L;
    if (!u) return;
    const ld *Bz = &ax[2].B[(e[2] * ax[2].nq + q[2]) * 3 * (ax[2].p + 1)];
    const ld *By = &ax[1].B[(e[1] * ax[1].nq + q[1]) * 3 * (ax[1].p + 1)];
    const ld *Bx = &ax[0].B[(e[0] * ax[0].nq + q[0]) * 3 * (ax[0].p + 1)];
    int pz = ax[2].p + 1, py = ax[1].p + 1, px = ax[0].p + 1;
    for (int az = 0; az < pz; ++az)
        for (int ay = 0; ay < py; ++ay)
            for (int ax0 = 0; ax0 < px; ++ax0) {
                long jz = e[2] + az, jy = e[1] + ay, jx = e[0] + ax0;
                ld c = (ld)u[(jz * ax[1].nb + jy) * ax[0].nb + jx];
                ld bx = Bx[ax0], by = By[ay], bz = Bz[az];
                ld dx = Bx[px + ax0], dy = By[py + ay], dz = Bz[pz + az];
                ld ddx = Bx[2 * px + ax0], ddy = By[2 * py + ay], ddz = Bz[2 * pz + az];
                *val += c * bx * by * bz;
                grad[0] += c * dx * by * bz;
                grad[1] += c * bx * dy * bz;
                grad[2] += c * bx * by * dz;
                *lap += c * (ddx * by * bz + bx * ddy * bz + bx * by * ddz);
            }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Petrov-Galerkin rows of the outer slab [r0, r1). */
static int rhs_pg(const or_problem *pb, const axis_t ax[3], const double *u, ld alpha, ld beta,
                  ld gamma, const or_source *src, long r0, long r1, double *b)
{
    const int o = pb->dim - 1; /* outermost real axis */
    long nrow[3], rlo[3], rhi[3], elo[3], ehi[3];
    for (int a = 0; a < 3; ++a) {
        nrow[a] = (a < pb->dim) ? pb->nspan[a] : 1;
        rlo[a] = 0;
        rhi[a] = nrow[a];
        elo[a] = 0;
        ehi[a] = ax[a].ne;
    }
    rlo[o] = r0;
    rhi[o] = r1;
    /* elements needed along the outer axis: the union of the slab's spans */
    elo[o] = ax[o].ne;
    ehi[o] = 0;
    for (long r = r0; r < r1; ++r) {
        long s, t;
        span_of(pb, o, r, &s, &t);
        if (s < elo[o]) elo[o] = s;
        if (t + 1 > ehi[o]) ehi[o] = t + 1;
    }
    long nel[3];
    for (int a = 0; a < 3; ++a) nel[a] = ehi[a] - elo[a];
    long nE = nel[0] * nel[1] * nel[2];
    ld *E = malloc(sizeof(ld) * (nE > 0 ? nE : 1));
    if (!E) return -2;

    /* element integrals with the test function equal to 1:
       E_e = sum_q W_q g(x_q),  g = alpha u_h + beta Lap u_h + gamma f */
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < nE; ++idx) {
        long e[3];
        e[0] = elo[0] + idx % nel[0];
        e[1] = elo[1] + (idx / nel[0]) % nel[1];
        e[2] = elo[2] + idx / (nel[0] * nel[1]);
        ld acc = 0.0L;
        int q[3];
        for (q[2] = 0; q[2] < ax[2].nq; ++q[2])
            for (q[1] = 0; q[1] < ax[1].nq; ++q[1])
                for (q[0] = 0; q[0] < ax[0].nq; ++q[0]) {
                    ld W = ax[0].W[e[0] * ax[0].nq + q[0]] * ax[1].W[e[1] * ax[1].nq + q[1]] *
                           ax[2].W[e[2] * ax[2].nq + q[2]];
                    ld val, grad[3], lap;
                    trial_at(ax, u, e, q, &val, grad, &lap);
                    ld g = alpha * val + beta * lap + gamma * source_at(pb, ax, src, e, q);
                    acc += W * g;
                }
        E[idx] = acc;
    }

    /* the integral over a span is the sum of its element integrals */
    long nR = (rhi[0] - rlo[0]) * (rhi[1] - rlo[1]) * (rhi[2] - rlo[2]);
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < nR; ++idx) {
        long r[3], w0 = rhi[0] - rlo[0], w1 = rhi[1] - rlo[1];
        r[0] = rlo[0] + idx % w0;
        r[1] = rlo[1] + (idx / w0) % w1;
        r[2] = rlo[2] + idx / (w0 * w1);
        long s[3], t[3];
        for (int a = 0; a < 3; ++a) span_of(pb, a, r[a], &s[a], &t[a]);
        ld acc = 0.0L;
        for (long ez = s[2]; ez <= t[2]; ++ez)
            for (long ey = s[1]; ey <= t[1]; ++ey)
                for (long ex = s[0]; ex <= t[0]; ++ex)
                    acc += E[((ez - elo[2]) * nel[1] + (ey - elo[1])) * nel[0] + (ex - elo[0])];
        b[idx] = (double)acc;
    }
    free(E);
    return 0;
}

/* Galerkin rows of the outer slab [r0, r1): loop over elements and Gauss
   points and add W * (test B_i) * integrand to the (p+1)^dim local rows. */
static int rhs_galerkin(const or_problem *pb, const axis_t ax[3], int form, const double *u,
                        ld alpha, ld beta, ld gamma, const or_source *src, long r0, long r1,
                        double *b)
{
    const int o = pb->dim - 1;
    long rlo[3], rhi[3], elo[3], ehi[3];
    for (int a = 0; a < 3; ++a) {
        rlo[a] = 0;
        rhi[a] = ax[a].nb;
        elo[a] = 0;
        ehi[a] = ax[a].ne;
    }
    rlo[o] = r0;
    rhi[o] = r1;
    /* B_i is nonzero on elements i-p .. i */
    elo[o] = r0 - pb->p < 0 ? 0 : r0 - pb->p;
    ehi[o] = r1 < ax[o].ne ? r1 : ax[o].ne;
    long w0 = rhi[0] - rlo[0], w1 = rhi[1] - rlo[1], w2 = rhi[2] - rlo[2];
    long nR = w0 * w1 * w2;
    ld *acc = calloc(nR > 0 ? nR : 1, sizeof(ld));
    if (!acc) return -2;
    long e[3];
    int q[3];
    for (e[2] = elo[2]; e[2] < ehi[2]; ++e[2])
        for (e[1] = elo[1]; e[1] < ehi[1]; ++e[1])
            for (e[0] = elo[0]; e[0] < ehi[0]; ++e[0])
                for (q[2] = 0; q[2] < ax[2].nq; ++q[2])
                    for (q[1] = 0; q[1] < ax[1].nq; ++q[1])
                        for (q[0] = 0; q[0] < ax[0].nq; ++q[0]) {
                            ld W = ax[0].W[e[0] * ax[0].nq + q[0]] *
                                   ax[1].W[e[1] * ax[1].nq + q[1]] *
                                   ax[2].W[e[2] * ax[2].nq + q[2]];
                            ld val, grad[3], lap;
                            trial_at(ax, u, e, q, &val, grad, &lap);
                            ld f = source_at(pb, ax, src, e, q);
                            const ld *Tx = &ax[0].B[(e[0] * ax[0].nq + q[0]) * 3 * (ax[0].p + 1)];
                            const ld *Ty = &ax[1].B[(e[1] * ax[1].nq + q[1]) * 3 * (ax[1].p + 1)];
                            const ld *Tz = &ax[2].B[(e[2] * ax[2].nq + q[2]) * 3 * (ax[2].p + 1)];
                            int px = ax[0].p + 1, py = ax[1].p + 1, pz = ax[2].p + 1;
                            for (int cz = 0; cz < pz; ++cz)
                                for (int cy = 0; cy < py; ++cy)
                                    for (int cx = 0; cx < px; ++cx) {
                                        long i[3] = {e[0] + cx, e[1] + cy, e[2] + cz};
                                        if (i[o] < r0 || i[o] >= r1) continue;
                                        ld test = Tx[cx] * Ty[cy] * Tz[cz];
                                        ld contrib;
                                        if (form == OR_GALERKIN_LAPLACIAN) {
                                            contrib = test * (alpha * val + beta * lap + gamma * f);
                                        } else {
                                            ld gtest[3] = {Tx[px + cx] * Ty[cy] * Tz[cz],
                                                           Tx[cx] * Ty[py + cy] * Tz[cz],
                                                           Tx[cx] * Ty[cy] * Tz[pz + cz]};
                                            contrib = test * (alpha * val + gamma * f) -
                                                      beta * (gtest[0] * grad[0] +
                                                              gtest[1] * grad[1] +
                                                              gtest[2] * grad[2]);
                                        }
                                        acc[((i[2] - rlo[2]) * w1 + (i[1] - rlo[1])) * w0 +
                                            (i[0] - rlo[0])] += W * contrib;
                                    }
                        }
    for (long k = 0; k < nR; ++k) b[k] = (double)acc[k];
    free(acc);
    return 0;
}

int or_rhs(const or_problem *pb, int form, const double *u, double alpha, double beta,
           double gamma, const or_source *src, long r0, long r1, double *b)
{
    if (form != OR_GALERKIN_BYPARTS && form != OR_GALERKIN_LAPLACIAN && form != OR_PG) return -1;
    if (check_problem(pb, form == OR_PG)) return -1;
    if (!b || (!u && (alpha != 0.0 || beta != 0.0))) return -1;
    const int o = pb->dim - 1;
    long nrow_o = (form == OR_PG) ? pb->nspan[o] : pb->ne[o] + pb->p;
    if (r0 < 0 || r1 > nrow_o || r0 >= r1) return -1;
    axis_t ax[3];
    int rc = build_axes(pb, ax);
    if (rc == 0) {
        if (form == OR_PG)
            rc = rhs_pg(pb, ax, u, alpha, beta, gamma, src, r0, r1, b);
        else
            rc = rhs_galerkin(pb, ax, form, u, alpha, beta, gamma, src, r0, r1, b);
    }
    for (int a = 0; a < 3; ++a) axis_free(&ax[a]);
    return rc;
}

int or_matrix_1d(int p, long ne, double lo, double hi, int nq, int kind, long nrows,
                 const long *span_first, const long *span_last, double *out)
{
    if (p < 1 || p > OR_MAXP || ne < 1 || !(lo < hi) || nq < 1 || nq > 64 || !out) return -1;
    long N = ne + p;
    int pg = (kind == OR_MAT_PG_MASS || kind == OR_MAT_PG_LAP);
    if (kind < 0 || kind > OR_MAT_PG_LAP) return -1;
    if (!pg && nrows != N) return -1;
    if (pg) {
        if (nrows < 1 || !span_first || !span_last) return -1;
        for (long r = 0; r < nrows; ++r)
            if (span_first[r] < 0 || span_last[r] < span_first[r] || span_last[r] >= ne) return -1;
    }
    axis_t ax;
    if (axis_build(&ax, p, ne, lo, hi, nq)) {
        axis_free(&ax);
        return -2;
    }
    ld *acc = calloc(nrows * N, sizeof(ld));
    if (!acc) {
        axis_free(&ax);
        return -2;
    }
    const int np = p + 1;
    if (!pg) {
        for (long e = 0; e < ne; ++e)
            for (int q = 0; q < nq; ++q) {
                long eq = e * nq + q;
                const ld *B = &ax.B[eq * 3 * np];
                ld W = ax.W[eq];
                for (int c = 0; c < np; ++c)      /* test  B_i, i = e + c */
                    for (int a = 0; a < np; ++a) { /* trial B_j, j = e + a */
                        ld v;
                        if (kind == OR_MAT_GAL_MASS)
                            v = B[c] * B[a];
                        else if (kind == OR_MAT_GAL_LAP)
                            v = B[c] * B[2 * np + a];
                        else
                            v = -B[np + c] * B[np + a];
                        acc[(e + c) * N + (e + a)] += W * v;
                    }
            }
    } else {
        for (long r = 0; r < nrows; ++r)
            for (long e = span_first[r]; e <= span_last[r]; ++e)
                for (int q = 0; q < nq; ++q) {
                    long eq = e * nq + q;
                    const ld *B = &ax.B[eq * 3 * np];
                    for (int a = 0; a < np; ++a) {
                        ld v = (kind == OR_MAT_PG_MASS) ? B[a] : B[2 * np + a];
                        acc[r * N + (e + a)] += ax.W[eq] * v;
                    }
                }
    }
    for (long k = 0; k < nrows * N; ++k) out[k] = (double)acc[k];
    free(acc);
    axis_free(&ax);
    return 0;
}

int or_explicit_step(const or_problem *pb, double *u, double dt, const or_source *src,
                     int nsteps)
{
    if (check_problem(pb, 1) || !u || nsteps < 0) return -1;
    /* the Petrov-Galerkin rows must be as many as the unknowns */
    for (int a = 0; a < pb->dim; ++a)
        if (pb->nspan[a] != pb->ne[a] + pb->p) return -1;
    const int o = pb->dim - 1;
    long n = 1;
    for (int a = 0; a < pb->dim; ++a) n *= pb->nspan[a];
    double *b = malloc(sizeof(double) * n);
    if (!b) return -2;
    /* |S_r| = product over the axes of the knot length t_{last+p+1} - t_{first+p} */
    ld *len[3] = {NULL, NULL, NULL};
    for (int a = 0; a < pb->dim; ++a) {
        knots_t kv = {pb->p, pb->ne[a], pb->lo[a], pb->hi[a]};
        len[a] = malloc(sizeof(ld) * pb->nspan[a]);
        for (long r = 0; r < pb->nspan[a]; ++r)
            len[a][r] = knot(&kv, pb->span_last[a][r] + pb->p + 1) -
                        knot(&kv, pb->span_first[a][r] + pb->p);
    }
    int rc = 0;
    for (int s = 0; s < nsteps && rc == 0; ++s) {
        rc = or_rhs(pb, OR_PG, u, 1.0, dt, dt, src, 0, pb->nspan[o], b);
        if (rc) break;
        long n0 = pb->nspan[0];
        long n1 = pb->dim > 1 ? pb->nspan[1] : 1;
        for (long k = 0; k < n; ++k) {
            ld m = len[0][k % n0];
            if (pb->dim > 1) m *= len[1][(k / n0) % n1];
            if (pb->dim > 2) m *= len[2][k / (n0 * n1)];
            u[k] = (double)((ld)b[k] / m);
        }
    }
    for (int a = 0; a < 3; ++a) free(len[a]);
    free(b);
    return rc;
}
