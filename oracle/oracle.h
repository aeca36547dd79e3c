/*
 * oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, direct CPU implementation of what the GPU library computes:
 * quadrature-based generation of isogeometric systems and right-hand sides for
 * C^{p-1} B-splines on open uniform knots (Paszynski, "Isogeometric analysis with
 * piece-wise constant test functions", arXiv:1910.08535), in the Galerkin form
 * (Section 1 and Section 2) and in the Petrov-Galerkin form whose test functions
 * are the indicators of spans of trial elements (Sections 2 and 3), plus the
 * forward-Euler explicit-dynamics step of Section 4.2.
 *
 * Only tests/, the smoke check of __graft_entry__ and the CPU-baseline leg of
 * bench.py may load this library.  It shares no code with the GPU library.
 * Every input and output is double; every sum is accumulated in long double.
 *
 * Conventions (0-based; the paper is 1-based):
 *   axis a in [0, dim): a = 0 is x (fastest in memory), a = 1 is y, a = 2 is z;
 *   axis a has ne[a] elements on [lo[a], hi[a]] and N_a = ne[a] + p B-splines;
 *   B_j is nonzero on elements max(0, j-p) .. min(ne-1, j);
 *   coefficient and row arrays are C-ordered (N_z, N_y, N_x), x fastest;
 *   a test span along an axis is an inclusive element range [first, last].
 */
#ifndef IGA_ORACLE_H
#define IGA_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAXP 8

/* forms of the generated rows */
enum { OR_GALERKIN_BYPARTS = 0, OR_GALERKIN_LAPLACIAN = 1, OR_PG = 2 };

/* 1D matrices of or_matrix_1d */
enum {
    OR_MAT_GAL_MASS = 0,     /* M(i,j)   =  int B_i B_j                           */
    OR_MAT_GAL_LAP = 1,      /* K(i,j)   =  int B_i B_j''   (Laplacian form)      */
    OR_MAT_GAL_BYPARTS = 2,  /* K(i,j)   = -int B_i' B_j'   (integrated by parts) */
    OR_MAT_PG_MASS = 3,      /* P(r,j)   =  int_{S_r} B_j                         */
    OR_MAT_PG_LAP = 4        /* P(r,j)   =  int_{S_r} B_j''                       */
};

typedef struct {
    int dim;                 /* 1, 2 or 3                                         */
    int p;                   /* degree, the same on every axis, 1 <= p <= OR_MAXP */
    long ne[3];              /* elements per axis                                 */
    double lo[3], hi[3];     /* domain per axis                                   */
    int nq[3];               /* Gauss points per element per axis                 */
    long nspan[3];           /* Petrov-Galerkin rows per axis                     */
    const long *span_first[3];
    const long *span_last[3];
} or_problem;

typedef struct {
    /* f(x) = sin_amp * prod_a sin(pi x_a) + table[q], both optional.  The table
       holds one value per Gauss point on the global Gauss grid of shape
       (ne_z*nq_z, ne_y*nq_y, ne_x*nq_x), x fastest; along an axis the point q of
       element e sits at e*nq + q, q ascending with the Gauss abscissa. */
    const double *table;
    double sin_amp;
} or_source;

/* Gauss-Legendre rule with nq points on [-1, 1], abscissae ascending. */
int or_gauss_legendre(int nq, double *xi, double *w);

/* Value (nder = 0) and derivatives up to nder <= 2 of every B-spline B_0..B_{N-1}
   of degree p on ne uniform elements of [lo, hi] at the point x.
   out[d*N + j] = d-th derivative of B_j at x.  Knot intervals are half-open
   [t_k, t_{k+1}) except the last, which is closed. */
int or_basis_eval(int p, long ne, double lo, double hi, double x, int nder, double *out);

/* Dense 1D matrix of kind OR_MAT_*, shape (nrows, N), row-major.  Galerkin kinds
   have nrows = N; Petrov-Galerkin kinds take one span per row. */
int or_matrix_1d(int p, long ne, double lo, double hi, int nq, int kind, long nrows,
                 const long *span_first, const long *span_last, double *out);

/* Rows of the generated right-hand side / operator apply:
     Galerkin:  b_i = sum_e sum_q W B_i(x_q) g(x_q)   (by-parts form replaces the
                B_i * beta*Lap(u_h) term by -beta*grad B_i . grad u_h)
     PG:        b_r = sum_{e in S_r} sum_q W g(x_q),  S_r = product of axis spans
   with g = alpha*u_h + beta*Lap(u_h) + gamma*f.  u may be NULL when alpha = beta = 0.
   Only rows whose outermost index lies in [r0, r1) are computed; they are stored
   contiguously in b (the slab), every other output value is untouched. */
int or_rhs(const or_problem *pb, int form, const double *u, double alpha, double beta,
           double gamma, const or_source *src, long r0, long r1, double *b);

/* nsteps forward-Euler steps of Section 4.2 in the Petrov-Galerkin form with the
   lumped left-hand side:  u <- [int_{S_r} (u_h + dt*Lap(u_h) + dt*f)] / |S_r|. */
int or_explicit_step(const or_problem *pb, double *u, double dt, const or_source *src,
                     int nsteps);

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
