/*
 * iga.h -- C ABI of the MI355X (gfx950) library for quadrature-based generation of
 * isogeometric systems and right-hand sides with C^{p-1} tensor-product B-splines
 * (Paszynski, "Isogeometric analysis with piece-wise constant test functions",
 * arXiv:1910.08535).
 *
 * Forms (Section 1, Section 2):
 *   IGA_GALERKIN_BYPARTS    test with B_i, Laplacian integrated by parts:
 *                           row i = int B_i (alpha u + gamma f) - beta int grad B_i . grad u
 *   IGA_GALERKIN_LAPLACIAN  test with B_i, not integrated by parts:
 *                           row i = int B_i (alpha u + beta Lap u + gamma f)
 *   IGA_PG                  Petrov-Galerkin form: the test function of row r is the
 *                           indicator of a span S_r of trial elements, obtained from
 *                           the Galerkin rows by summing the rows of the B-splines that
 *                           are nonzero on the span (partition of unity), so that the
 *                           test function is never evaluated (Section 2, Section 3):
 *                           row r = int_{S_r} (alpha u + beta Lap u + gamma f)
 *   Operator IGA_OP_LAPLACE is +Lap in every form (the caller negates for -Lap u = f,
 *   Section 4.3).
 *
 * Conventions.
 *   - Axis a in [0, dim): a = 0 is x, a = 1 is y, a = 2 is z.  Axis a has ne[a]
 *     uniform elements on [lo[a], hi[a]], an open knot vector, and N_a = ne[a] + p
 *     B-splines (Section 2).  B_j is nonzero on elements max(0,j-p) .. min(ne-1,j).
 *   - Coefficient arrays u and row arrays b are C-ordered (N_z, N_y, N_x) /
 *     (R_z, R_y, R_x), x fastest, FP64, contiguous (Section 3 and 4.1 number the
 *     unknowns with x fastest).  R_a = N_a for Galerkin forms and for PG spans
 *     IGA_SPANS_SUPPORT; R_a = ne[a] for IGA_SPANS_ELEMENT; R_a = nspan[a] for
 *     IGA_SPANS_CUSTOM.
 *   - PG spans (inclusive element ranges [first, last] per row and axis; the tensor
 *     span is the product of the axis spans):
 *       IGA_SPANS_SUPPORT  S_r = supp B_r = [max(0,r-p), min(ne-1,r)] -- every element
 *                          integral is added to the p+1 rows of the B-splines living on
 *                          it, as in the piece-wise-constant generation loops of
 *                          Section 4.1 and Section 4.3;
 *       IGA_SPANS_ELEMENT  S_e = {e} -- the single-element integrals (the rows of the
 *                          worked example of Section 2 where p+1 consecutive B-splines
 *                          sum to one);
 *       IGA_SPANS_CUSTOM   caller tables; each S_r must lie inside supp B_r;
 *       IGA_SPANS_REFINED  the refined test space (Section 2): every trial element of axis
 *                          a is split into refine[a] elements, and row i sums the test
 *                          B-splines of degree p on those refined open knots whose sum is
 *                          1 on the row's cell and ramps over p refined elements on each
 *                          side; the cells partition the axis at the midpoints of
 *                          consecutive Greville abscissae (rounded to refined element
 *                          boundaries).  The system is square (R_a = N_a) and regular, its
 *                          rows are integrated with nq[a] Gauss points on every refined
 *                          element, and iga_solve accepts it.
 *   - Gauss rule: nq[a] Gauss-Legendre points per element on axis a; weight times
 *     Jacobian W = w h / 2 per axis (Section 2, Section 4.1).
 *   - A source f is   sin_amp * prod_a sin(pi x_a)   plus an optional table with one
 *     value per Gauss point on the global Gauss grid, shape
 *     (ne_z nq_z, ne_y nq_y, ne_x nq_x), x fastest, point q of element e at e*nq + q
 *     with q ascending in the abscissa.
 *
 * Memory and execution.
 *   - Every array argument is a DEVICE pointer owned by the caller, except where
 *     marked "host".  The library never frees caller memory.  A context owns its
 *     tables and its scratch buffers only.
 *   - Calls enqueue kernels on the context's HIP stream and return without waiting
 *     (asynchronous); argument errors are detected and returned before anything is
 *     enqueued.  One context per stream; calls on one context are not thread-safe.
 *   - A call that would allocate device memory (context creation, the scratch of a
 *     first call that needs it, the tables of a first solve) returns IGA_E_INVAL while
 *     the context's stream is being captured into a graph; calls after it can be
 *     captured.
 *   - Return value: IGA_OK (0) or a negative IGA_E_* code; nothing throws.
 *   - All arithmetic is FP64.
 */
#ifndef IGA_H
#define IGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IGA_OK 0
#define IGA_E_INVAL (-1)       /* bad argument (null pointer, size, range, span table) */
#define IGA_E_UNSUPPORTED (-2) /* dim not in {1,2,3}, p not in {2,3}, nq not in [1,16];  */
                               /* a Gauss-point table source or boundary terms with      */
                               /* refined PG rows                                        */
#define IGA_E_NOMEM (-3)       /* device allocation failed / batch over its memory budget */
#define IGA_E_DEVICE (-4)      /* a HIP call failed */
#define IGA_E_AGAIN (-5)       /* batch queue full: poll and submit again */
#define IGA_E_SINGULAR (-6)    /* solve with the Petrov-Galerkin form (singular system)  */

typedef enum { IGA_GALERKIN_BYPARTS = 0, IGA_GALERKIN_LAPLACIAN = 1, IGA_PG = 2 } iga_form;
typedef enum { IGA_OP_MASS = 0, IGA_OP_LAPLACE = 1 } iga_op;
typedef enum { IGA_SPANS_SUPPORT = 0, IGA_SPANS_ELEMENT = 1, IGA_SPANS_CUSTOM = 2, IGA_SPANS_REFINED = 3 } iga_spans;

typedef struct {
    int32_t dim;        /* 1, 2 or 3                                                  */
    int32_t p;          /* B-spline degree on every axis: 2 (C1) or 3 (C2)             */
    int64_t ne[3];      /* elements per axis, >= 1 (entries beyond dim ignored); at    */
                        /* most 2^31-1 coefficients in all; in 2D every array and band */
                        /* table below 4 GiB: N_x N_y < 2^29, N_a (2p+1) < 2^29; in 3D */
                        /* one plane below 4 GiB: N_x N_y < 2^29                       */
    double lo[3];       /* domain per axis, lo < hi                                    */
    double hi[3];
    int32_t nq[3];      /* Gauss points per element per axis, 1..16                    */
    int32_t spans;      /* iga_spans                                                   */
    /* IGA_SPANS_CUSTOM only (host, read during iga_create and not kept):             */
    int64_t nspan[3];
    const int64_t *span_first[3];
    const int64_t *span_last[3];
    /* IGA_SPANS_REFINED only: refined elements per trial element, 1..64 per axis; the    */
    /* cells must be non-empty and every row's columns within r-p .. r+p (refine >= 4     */
    /* always qualifies for p = 2, 3)                                                     */
    int32_t refine[3];
} iga_mesh_desc;

typedef struct {
    const double *table; /* device, nullable: one value per Gauss point (layout above) */
    double sin_amp;      /* amplitude of prod_a sin(pi x_a); 0 for none                */
} iga_source;

typedef struct iga_ctx iga_ctx;

/* Creates a context for one mesh: validates the descriptor and builds, with device
   kernels, the per-axis Gauss rule, the basis tables and the banded 1D factors.
   hip_stream: a hipStream_t (NULL = the default stream) on which every call of this
   context is enqueued.  The set-up kernels are enqueued on that stream too (every later
   call of the context is ordered after them); only caller span tables (CUSTOM) are
   copied synchronously.  The tables of an axis depend only on (p, ne, nq, lo, hi, span
   kind): contexts with equal axes share one copy (built once, on the stream of the first
   context that needs it; later contexts' streams wait for that build), and tables no
   context uses stay cached up to 4 GiB per device, least recently released first out.
   Device memory comes from the device's default stream-ordered pool; the first call on
   a device sets that pool to keep freed memory (no release threshold) so that contexts
   can be created and destroyed at a high rate.  Contexts must not be created from
   several host threads at once.
   Errors: IGA_E_INVAL (null out, bad sizes or spans), IGA_E_UNSUPPORTED,
   IGA_E_NOMEM, IGA_E_DEVICE. */
int iga_create(const iga_mesh_desc *desc, void *hip_stream, iga_ctx **out);

/* Releases the context's tables, scratch and cached graph.  Device memory is freed in
   stream order (after the work already queued on the context's stream), so this does
   not wait, except for a cached explicit-step graph, which is waited for first. */
int iga_destroy(iga_ctx *ctx);

/* Row counts R_a (rows, host, [3]) of `form` and basis counts N_a (cols, host, [3]);
   entries beyond dim are 1. */
int iga_shape(const iga_ctx *ctx, int32_t form, int64_t rows[3], int64_t cols[3]);

/* System matrices as banded 1D factors (Section 4.1: the tensor-product matrices are
   Kronecker products of 1D matrices, the structure used by the alternating-directions
   solver).  Writes `bands` (device, caller-allocated, dim*2*Rmax*(2p+1) doubles,
   Rmax = max_a R_a): bands[((a*2 + f)*Rmax + r)*(2p+1) + k] is the entry of factor f
   on axis a in row r, column r + k - p (zero where that column does not exist and in
   rows r >= R_a).  Factor 0 is the mass-type factor (Galerkin: int B_r B_j; PG:
   int_{S_r} B_j); factor 1 is the operator factor (Galerkin Laplacian form:
   int B_r B_j''; by parts: -int B_r' B_j'; PG: int_{S_r} B_j'').
   The d-dimensional matrix is  MASS: prod_a F0_a  and  LAPLACE: sum_t prod_a
   (a == t ? F1_a : F0_a)  (Kronecker products, x fastest).  `op` selects whether
   factor 1 is written (IGA_OP_LAPLACE) or left untouched (IGA_OP_MASS).
   Errors: IGA_E_INVAL. */
int iga_assemble(iga_ctx *ctx, int32_t form, int32_t op, double *bands);

/* Right-hand side / operator application (Section 2-4.1):
     b_r = int T_r (alpha u_h + beta Lap u_h + gamma f)
   with T_r = B_r (Galerkin forms) or the indicator of S_r (PG), u_h = sum_j u_j B_j.
   u: device coefficients (N_z,N_y,N_x), may be NULL when alpha = beta = 0.
   f: host struct (NULL = no source); its table is a device pointer.
   b: device rows (R_z,R_y,R_x), must not alias u or f->table.
   Errors: IGA_E_INVAL. */
int iga_rhs(iga_ctx *ctx, int32_t form, const double *u, double alpha, double beta,
            double gamma, const iga_source *f, double *b);

/* Fused matrix-free application of both operators in one pass over u:
     mass_out_r = int T_r u_h,   lap_out_r = int T_r Lap u_h   (by parts for
   IGA_GALERKIN_BYPARTS).  Either output may be NULL (not both).
   Errors: IGA_E_INVAL. */
int iga_apply(iga_ctx *ctx, int32_t form, const double *u, double *mass_out, double *lap_out);

/* nsteps forward-Euler steps of u_t = Lap u + f (Section 4.2) in the PG form with
   support spans, the left-hand side lumped by its row sums (partition of unity:
   sum_j int_{S_r} B_j = |S_r|):
     u_r <- int_{S_r} (u_h + dt Lap u_h + dt f) / |S_r|.
   u: device coefficients, updated in place.  Requires IGA_SPANS_SUPPORT (square
   system).  For nsteps >= 2, the second consecutive call with the same
   (u, dt, f, nsteps) captures the launches into a HIP graph that is cached on the
   context and replayed while they stay the same (a first call launches directly).
   Errors: IGA_E_INVAL (also for other span kinds), IGA_E_NOMEM. */
int iga_explicit_step(iga_ctx *ctx, double *u, double dt, const iga_source *f, int32_t nsteps);

/* For callers that cannot allocate device memory (code under graph capture, tight serving
   loops, harnesses that forbid hipMalloc): iga_explicit_step with the same kernels and
   results, bit for bit, that allocates nothing.  The steps ping-pong between u and a work
   buffer that is a static device array of the library, IGA_NOALLOC_MAX_DOUBLES doubles
   (64 MiB) on every device the library runs on, held until the process ends; the call
   launches directly (no graph is cached).  Every call on a device shares that device's
   array, which keeps the last call's contents: calls that overlap on one device (other
   streams, other threads, other contexts) race and must be ordered by the caller.
   Sources: sin_amp only; a Gauss-point table gives IGA_E_UNSUPPORTED.
   Errors: IGA_E_INVAL (as iga_explicit_step), IGA_E_UNSUPPORTED (table source),
   IGA_E_NOMEM (more than IGA_NOALLOC_MAX_DOUBLES coefficients), IGA_E_DEVICE. */
#define IGA_NOALLOC_MAX_DOUBLES ((size_t)1 << 23)
int iga_explicit_step_noalloc(iga_ctx *ctx, double *u, double dt, const iga_source *f, int32_t nsteps);

/* Alternating-directions direct solve with the Galerkin mass (Section 4.1):
     (M_z (x) M_y (x) M_x) x = b,   M_a(i, j) = int B_i B_j  on axis a,
   the matrix of the Galerkin L2 projection.  The Kronecker structure reduces it to
   three families of 1D banded systems with many right-hand sides: along x for every
   (y, z) line, then along y, then along z.  Each M_a (bandwidth p, symmetric positive
   definite) is factorized once, M_a = L_a L_a^T, at the context's first solve (kernels
   on its stream; the factors stay with the context), and every solve runs a forward and
   a backward substitution along every line.  Axes with few lines (1D, and 2D up to a
   few thousand lines) are solved in chunks instead: the chunks' own factors, the
   coupling between neighbouring chunks and a small block system per line, all built
   once per context, give the same solution to rounding.  When the coupling between
   neighbouring chunk boundaries is below 2^-64 (it decays geometrically along a chunk),
   the block system is taken as block diagonal; deciding this reads one small table back
   to the host at the context's first solve along the axis (one synchronisation of its
   stream; with the context setting IGA_TILE_SOLVE_EXACT = 1 (iga_set_tile) the full
   block system is always used and nothing is read back; iga_solve_info reports the
   choice).
   The first solve of a context allocates and builds these tables, so it must not be
   captured into a graph (IGA_E_INVAL while the context's stream is capturing); once it
   has run, solves can be captured and replayed.
   b, x: device coefficient arrays (N_z, N_y, N_x); x may equal b (in place); b is not
   modified unless x == b.  form: IGA_GALERKIN_BYPARTS or IGA_GALERKIN_LAPLACIAN (one
   mass matrix for both).
   With IGA_PG on a context with IGA_SPANS_REFINED spans the solve uses the square PG
   mass factors [int T_i B_j] of the refined test space instead (banded LU without
   pivoting, once per context).
   Errors: IGA_E_INVAL, IGA_E_SINGULAR for IGA_PG with spans made of whole elements (the
   PG mass matrix then has rank at most prod_a ne[a] < prod_a N_a), IGA_E_NOMEM. */
int iga_solve(iga_ctx *ctx, int32_t form, const double *b, double *x);

/* How the solves along axis `axis` (0 = x) of a context run, as chosen at its first solve
   (host outputs, nullable): *scheme is
     IGA_SOLVE_NONE            no solve has run on the context yet;
     IGA_SOLVE_LINES           one forward and one backward recurrence along every line;
     IGA_SOLVE_PART_EXACT      partitioned into *chunks chunks per line, the small block
                               system that couples the chunks solved exactly along the line;
     IGA_SOLVE_PART_BLOCKDIAG  partitioned, that block system taken as block diagonal (its
                               dropped coupling below 2^-64, as described at iga_solve).
   Reads host state only; never blocks.  Errors: IGA_E_INVAL (null ctx, axis outside
   [0, dim)). */
#define IGA_SOLVE_NONE 0
#define IGA_SOLVE_LINES 1
#define IGA_SOLVE_PART_EXACT 2
#define IGA_SOLVE_PART_BLOCKDIAG 3
int iga_solve_info(const iga_ctx *ctx, int32_t axis, int32_t *scheme, int32_t *chunks);

/* nsteps forward-Euler steps of u_t = Lap u + f (Section 4.2) in a Galerkin form with
   the consistent mass:
     M u_{t+1} = int B_r (u_t + dt Lap u_t + dt f)   (Laplacian term by parts for
   IGA_GALERKIN_BYPARTS),
   the right-hand side generated as by iga_rhs and the mass system solved as by
   iga_solve.  With IGA_PG on a context with refined spans the same step is taken with
   the refined test functions and their square mass.  u: device coefficients, updated in
   place.  The scheme is stable only for dt below 2 / lambda_max(M^{-1} K) (of order h^2).
   Errors: IGA_E_INVAL, IGA_E_SINGULAR for IGA_PG with spans of whole elements,
   IGA_E_NOMEM. */
int iga_galerkin_step(iga_ctx *ctx, int32_t form, double *u, double dt, const iga_source *f,
                      int32_t nsteps);

/* A side of the domain for boundary conditions: side = 2a is the lower end of axis a,
   2a + 1 its upper end.  The Neumann datum G on the side is g_const plus, when g_table
   is given (device), one value per Gauss point of the side: the side's elements and
   Gauss points along its tangential axes, taken in increasing axis order with the first
   fastest (1D: one value). */
typedef struct {
    int32_t side;
    const double *g_table;
    double g_const;
} iga_side;

/* Boundary terms of the Laplace problem with mixed conditions (Section 4.3): after the
   Laplacian is integrated back by parts, a Neumann side G carries
     b_r += alpha int_G T_r du_h/dn dS + beta int_G T_r G dS
   with T_r = B_r (Galerkin forms) or the indicator of the span S_r (PG), n the outward
   normal, for every listed side, added to b (device rows, as written by iga_rhs).
   With the Laplacian form the system of the problem -Lap u = f, du/dn = G on the
   Neumann sides reads  -iga_apply(lap) + (alpha = 1 term) = iga_rhs(f) + (beta = 1 term)
   (the by-parts form already carries the boundary integral of every side).
   sides: host array of nsides entries; u: device coefficients (needed when alpha != 0);
   b must not alias u or a table.  Errors: IGA_E_INVAL. */
int iga_boundary_terms(iga_ctx *ctx, int32_t form, int32_t nsides, const iga_side *sides,
                       const double *u, double alpha, double beta, double *b);

/* Zero Dirichlet conditions by row replacement (Section 4.3): the rows of the B-splines
   that do not vanish on a listed side (bit 2a of side_mask: lower end of axis a, bit
   2a + 1: upper end; under open knots B_0 and B_{N-1} of that axis) become identity rows:
   rows[r] = u[r] (the operator applied to u), or 0 when u is NULL (the right-hand side).
   Square systems only: Galerkin forms, or PG with support spans.
   Errors: IGA_E_INVAL. */
int iga_dirichlet_rows(iga_ctx *ctx, int32_t form, int32_t side_mask, const double *u, double *rows);

/* Tile configuration of the context's kernels (what the autotuner varies).  A setting
   fixes the order of every sum, so results are reproducible for a given setting; other
   settings differ from it by round-off only.  Keys:
     IGA_TILE_2D_ROWS    output rows per 2D wave chunk of 128 columns: 2, 4, 8 (default) or 16
     IGA_TILE_2D_ORDER   2D chunk order: 0 = XCD-aware, row bands first (default);
                         1 = XCD-aware, strips first; 2 = plain dispatch order
     IGA_TILE_3D_PLANES  output planes per 3D z-chunk: 1..32, 0 = automatic (default)
     IGA_TILE_3D_ROWS    output rows per 3D tile: even, 2..32, 0 = automatic (default;
                         fewer when the tile's footprint would not fit a workgroup)
     IGA_TILE_3D_COLS    output columns per 3D tile: even, 8..96, 0 = automatic (default)
     IGA_TILE_2D_STRIP   2D strip width: 128 columns, two per lane (default), or 64, one
                         per lane (same bits)
     IGA_TILE_SOLVE_EXACT  partitioned solves (iga_solve): 0 = the block system that couples
                         the chunks taken as block diagonal where its dropped coupling is
                         below 2^-64 (default), 1 = always solved whole (no read-back at the
                         first solve); accepted only before the context's first solve
   Changing a launch setting drops the context's cached graph.
   Errors: IGA_E_INVAL (unknown key or value; IGA_TILE_SOLVE_EXACT after a solve). */
#define IGA_TILE_2D_ROWS 1
#define IGA_TILE_3D_PLANES 2
#define IGA_TILE_3D_ROWS 4
#define IGA_TILE_2D_ORDER 5
#define IGA_TILE_3D_COLS 6
#define IGA_TILE_2D_STRIP 7
#define IGA_TILE_SOLVE_EXACT 8
int iga_set_tile(iga_ctx *ctx, int32_t key, int32_t value);
int iga_get_tile(const iga_ctx *ctx, int32_t key, int32_t *value);

/* Autotuning of a 2D or 3D context's tile setting.  Times every candidate setting of the
   hot kernel of op -- IGA_TUNE_APPLY: the fused PG apply (mass and Laplacian rows, as
   iga_apply); IGA_TUNE_STEP: one lumped explicit step with a sine source (as
   iga_explicit_step) -- with reps >= 1 launches each after two warm-up launches, on
   buffers of its own (enough sets, used in turn, to exceed twice the 256 MB Infinity Cache,
   at most 32: the launches read and write HBM), timed with HIP events on the context's
   stream (two rounds over the
   candidates, the better round of each counting).  The fastest setting becomes the
   context's -- unless the setting the context had is a candidate within 3% of it, which
   then stays -- and the process remembers it: contexts created later with the
   same dim, p, span kind and size class (the bit length of every axis' row count) start
   from it.  Candidates, in this order (times_us follows it):
     2D: IGA_TILE_2D_STRIP in {128, 64} x IGA_TILE_2D_ROWS in {4, 8, 16}
         x IGA_TILE_2D_ORDER in {0, 1}                                   (12)
     3D: IGA_TILE_3D_PLANES in {0, 6, 12} x IGA_TILE_3D_ROWS in {0, 8}
         x IGA_TILE_3D_COLS in {0, 32}                                   (12)
   Every candidate forms every sum in the same order, so the results do not depend on the
   choice.  Blocks until its launches are done.  A 1D context has nothing to tune: IGA_OK
   with *ntimed = 0.  times_us (nullable, IGA_TUNE_MAX entries) receives the average
   microseconds per launch of each candidate, *ntimed (nullable) their number.
   Errors: IGA_E_INVAL (bad op or reps, stream capture, a span kind without the op),
   IGA_E_NOMEM, IGA_E_DEVICE. */
#define IGA_TUNE_APPLY 0
#define IGA_TUNE_STEP 1
#define IGA_TUNE_MAX 16
int iga_autotune(iga_ctx *ctx, int32_t op, int32_t reps, float *times_us, int32_t *ntimed);

/* Bandwidth reference of the fused 2D apply (not part of the method): reads the n doubles
   of src once and writes them to dst_a and dst_b (device, caller-owned, no overlap), with
   the 16-byte accesses and streaming stores of the apply kernel, on hip_stream (NULL =
   default stream).  Its time is the floor a launch moving the same bytes can reach.
   Errors: IGA_E_INVAL (null pointer, n = 0 or n >= 2^29). */
int iga_copy_probe(const double *src, double *dst_a, double *dst_b, size_t n, void *hip_stream);

/* Error string of an IGA_* code (static storage). */
const char *iga_strerror(int code);

/* ---------------------------------------------------------------------------------
 * Batched execution: many independent 2D problems of different sizes and degrees in
 * ONE persistent kernel launch (captured once into a HIP graph and replayed), whose
 * waves claim chunks of rows from a device work counter.  Every job is the fused
 * Petrov-Galerkin apply of iga_apply (mass rows and Laplacian rows, support spans) on
 * its own space: p in {2,3}, ne[0] x ne[1] elements on [0,1]^2, p+1 Gauss points per
 * axis.  Per-mesh tables are built once and cached in the batch.  Results are identical,
 * bit for bit, to iga_apply on a context with the same tile setting.
 * ------------------------------------------------------------------------------ */
typedef enum { IGA_JOB_QUEUED = 0, IGA_JOB_RUNNING = 1, IGA_JOB_DONE = 2, IGA_JOB_FAILED = 3 } iga_job_state;

typedef struct {
    int32_t p;          /* 2 or 3                                                       */
    int64_t ne[2];      /* elements along x and y, >= 1                                  */
    const double *u;    /* device coefficients, shape (ne[1]+p, ne[0]+p), x fastest      */
    double *mass_out;   /* device rows int_{S_r} u_h, same shape                         */
    double *lap_out;    /* device rows int_{S_r} Lap u_h, same shape                     */
} iga_job;

typedef struct iga_batch iga_batch;

/* hip_stream: stream of every batch launch (NULL = default stream).
   mem_budget_bytes: admission limit on the bytes the queued and running jobs touch
   (u and both outputs); 0 = unlimited.  max_jobs: jobs per launch (queue capacity).
   Errors: IGA_E_INVAL, IGA_E_NOMEM, IGA_E_DEVICE. */
int iga_batch_create(void *hip_stream, size_t mem_budget_bytes, int32_t max_jobs,
                     iga_batch **out);
/* Validates and queues njobs jobs (host array); tickets (host, [njobs]) receive their
   ids.  All or nothing: IGA_E_INVAL for a bad job, IGA_E_UNSUPPORTED for p outside
   {2,3}, IGA_E_AGAIN when the queue or the memory budget cannot take all of them now
   (poll or wait, then submit again). */
int iga_batch_submit(iga_batch *b, const iga_job *jobs, int32_t njobs, uint64_t *tickets);
/* Launches one persistent kernel over the queued jobs (asynchronous).  A launch still
   running is waited for first, so jobs that arrive while one launch runs ride the
   next.  No-op when nothing is queued. */
int iga_batch_flush(iga_batch *b);
/* state (host): IGA_JOB_QUEUED / RUNNING / DONE / FAILED of a ticket.  The jobs of one
   launch complete together (the launch's HIP event); never blocks.  IGA_E_INVAL:
   unknown ticket. */
int iga_batch_poll(iga_batch *b, uint64_t ticket, int32_t *state);
/* Blocks until the running launch, if any, is done. */
int iga_batch_wait(iga_batch *b);
/* Autotuner: times the queued jobs (which stay queued; applies are idempotent) with
   every chunk height of the 2D kernel: the job list is uploaded once per height, then
   `reps` launches of the persistent kernel are timed with HIP events on the batch stream
   (the launches only, no host work or copy between them).  Keeps the fastest height for
   later launches and writes it to best_rows and its time per launch in milliseconds to
   best_ms (host, both nullable).  Blocks until the timed launches are done. */
int iga_batch_autotune(iga_batch *b, int32_t reps, int32_t *best_rows, float *best_ms);
int iga_batch_destroy(iga_batch *b);

/* ---------------------------------------------------------------------------------
 * Serving: a request loop inside the library, for a stream of independent requests on
 * meshes of any size.  A request is either
 *   IGA_REQ_RHS   the fused Petrov-Galerkin apply of iga_apply (mass and Laplacian rows,
 *                 support spans), or
 *   IGA_REQ_STEP  nsteps explicit steps of iga_explicit_step (u updated in place) with a
 *                 source sin_amp * prod_a sin(pi x_a),
 * on dim axes of ne[a] elements on [0, 1], degree p, p+1 Gauss points per axis.
 * Requests are admitted in submission order while the bytes of the requests in flight
 * stay within the budget: u and both outputs, or u and the step's work buffer, plus a
 * batched request's own band tables (M and D rows per axis and the step's scale and
 * source rows; in 1D only the step's source rows).  A request whose every axis has at
 * least 3p+1 elements is batched: it needs no context, and all admitted batched requests
 * advance together in iterations, each one descriptor copy and one launch per kind of
 * request (1D, 2D, 3D per degree and kind) on the server's own streams, at most two
 * iterations in flight.  A right-hand side runs in one iteration, a step request takes
 * one step per iteration (continuous batching at the granularity of a step); a request
 * admitted while iterations run joins the next one.  Any other request runs at once on
 * the stream of its mesh's context: contexts are cached (least recently used first out
 * while the device memory the cached contexts hold -- their tables and scratch, such as
 * an explicit step's work buffer -- exceeds cache_bytes; the most recently used one
 * always stays) and bound round-robin to the server's streams.  Completion is observed
 * from HIP events; no call blocks except iga_server_destroy.  Results equal those of the
 * same request run alone through iga_apply / iga_explicit_step, bit for bit.  All
 * buffers are caller-owned device memory and must stay valid until the request is
 * reported done.
 * ------------------------------------------------------------------------------ */
#define IGA_REQ_RHS 0
#define IGA_REQ_STEP 1

typedef struct {
    int32_t kind;          /* IGA_REQ_RHS or IGA_REQ_STEP                               */
    int32_t dim, p;        /* 1..3; 2 or 3                                              */
    int64_t ne[3];         /* elements per axis (x, y, z), >= 1                          */
    int32_t nsteps;        /* STEP: steps, >= 1                                          */
    double dt, sin_amp;    /* STEP: time step, source amplitude                          */
    double *u;             /* device coefficients (N_z, N_y, N_x); STEP: updated         */
    double *mass_out;      /* RHS: device rows, same shape as u                          */
    double *lap_out;       /* RHS: device rows, same shape as u                          */
} iga_request;

typedef struct iga_server iga_server;

/* nstreams (1..64) streams of default priority; mem_budget_bytes > 0; cache_bytes:
   limit on the device bytes of the cached contexts (tables and scratch).
   Errors: IGA_E_INVAL, IGA_E_NOMEM. */
int iga_server_create(int32_t nstreams, size_t mem_budget_bytes, size_t cache_bytes,
                      iga_server **out);
/* Queues n requests (host array; all or nothing) and admits what fits; tickets (host,
   [n]) receive their ids.  Errors: IGA_E_INVAL (bad request), IGA_E_UNSUPPORTED (dim or
   p), IGA_E_NOMEM (a request larger than the whole budget). */
int iga_server_submit(iga_server *s, const iga_request *reqs, int32_t n, uint64_t *tickets);
/* Harvests completions, admits queued requests that now fit and enqueues iterations while
   fewer than two are in flight and batched requests have work left; then reports up to
   cap completed requests (host arrays): ticket, time in seconds since the server was
   created (when the completion was observed), state (IGA_JOB_DONE or IGA_JOB_FAILED) and,
   if done_launch is not NULL, the index of the iteration that ran its last kernel (-1 for
   a request run on a context).  *ndone receives the count.  Never blocks.  Errors:
   IGA_E_INVAL; IGA_E_DEVICE (a HIP call failed: the server can only be destroyed). */
int iga_server_progress(iga_server *s, uint64_t *done, double *done_time, int32_t *done_state,
                        int64_t *done_launch, int32_t cap, int32_t *ndone);
/* Bytes in flight, their peak, iterations enqueued so far (batch_launches), and the
   server's clock (seconds since creation); every output is nullable. */
int iga_server_stats(const iga_server *s, size_t *used, size_t *peak, int64_t *batch_launches,
                     double *now);
/* Device bytes held by the cached contexts (tables and scratch, as counted against
   cache_bytes) and their number; both outputs nullable. */
int iga_server_cache_stats(const iga_server *s, size_t *cache_bytes, int64_t *contexts);
/* Waits for the server's streams, then releases its contexts, streams and events. */
int iga_server_destroy(iga_server *s);

#ifdef __cplusplus
}
#endif
#endif /* IGA_H */
