// Partitioned solve of one family of lines of the alternating-directions solve
// (Section 4.1), for families with few lines (1D, and 2D up to a few thousand lines per
// family), where one recurrence per line leaves most of the GPU idle.
//
// The 1D matrix A (n x n, bandwidth P, the same for every line of the family) is cut into
// K chunks of rows [s_k, e_k), e_k = s_{k+1}, of at least 64 >= 2P rows each (PartGeom):
// balanced, s_k = floor(k n / K), or, for a single line, interior chunks of exactly m rows
// between a first and a last chunk (of 16 or more rows), so that the interior chunks have
// bitwise equal factors and run as the lines of one segment-kernel launch.  With D the
// block diagonal of the chunks' own blocks A_kk,
// A = D (I + S), and the spikes of S are line-independent:
//     V_k = A_kk^{-1} A(chunk k, first P columns of chunk k+1)     (e_k - s_k) x P
//     W_k = A_kk^{-1} A(chunk k, last P columns of chunk k-1)      (e_k - s_k) x P
// A line's solve is then
//   1. g = D^{-1} b: independent solves of every chunk of every line (LU factors of the
//      chunks, in the sweep-table format of the other solves, so that the segment kernel
//      runs them, one chunk per workgroup row, when there are lines enough to fill its
//      lanes);
//   2. the reduced system in zeta_k = (u_k, t_{k+1}), u_k the last P values of chunk k and
//      t_{k+1} the first P of chunk k+1 (k = 0 .. K-2):
//          u_k + V_k^B t_{k+1} + W_k^B u_{k-1} = g_k^B,
//          t_{k+1} + W_{k+1}^T u_k + V_{k+1}^T t_{k+2} = g_{k+1}^T
//      (^T: first P rows of a spike, ^B: last P rows), block tridiagonal with 2P x 2P
//      blocks D_k = [I, V_k^B; W_{k+1}^T, I], E_k = [W_k^B, 0; 0, 0] below and
//      F_k = [0, 0; 0, V_{k+1}^T] above the diagonal.  Its block LU is line-independent:
//      Delta_0 = D_0, Gamma_k = E_k Delta_{k-1}^{-1}, Delta_k = D_k - Gamma_k F_{k-1}; per
//      line a forward sweep y_k = h_k - Gamma_k y_{k-1} (h_k = (g_k^B, g_{k+1}^T)) and a
//      backward sweep zeta_k = Delta_k^{-1} (y_k - F_k zeta_{k+1});
//   3. x = g - V_k t_{k+1} - W_k u_{k-1} on every row of chunk k.
// This is exact (no truncation of the spikes), so it agrees with the sequential solve to
// rounding.  The spikes decay fast away from the chunk ends (for the mass matrices of
// this method Gamma is below 1e-16 for chunks of 64 rows), so the reduced system is well
// conditioned.  Where the entries of E_k and F_k are all below 2^-64 (chunks of about 50
// rows for p = 2, 70 for p = 3), dropping them changes no value of zeta by more than a
// small fraction of its last bit; step 2 then solves every interface on its own, inside
// the correction (part_fix_kernel), instead of the sweeps along the line.
#pragma once
#include "ads.hpp"
#include "common.hpp"

namespace iga {

// Chunk geometry.  m = 0: balanced chunks, s_k = floor(k n / K) in 32-bit arithmetic
// (the host keeps (K + 1) n below 2^32).  m > 0: s_0 = 0, s_k = f + (k-1) m for
// 0 < k < K, s_K = n.
struct PartGeom {
    int n, K, f, m;
    __host__ __device__ int start(int k) const
    {
        if (m == 0) return (int)((unsigned)k * (unsigned)n / (unsigned)K);
        return k <= 0 ? 0 : (k >= K ? n : f + (k - 1) * m);
    }
    // the chunk of row r: s_k <= r < s_{k+1}
    __host__ __device__ int chunk(int r) const
    {
        if (m == 0) return (int)(((unsigned)(r + 1) * (unsigned)K + (unsigned)n - 1u) / (unsigned)n) - 1;
        return r < f ? 0 : min(1 + (r - f) / m, K - 1);
    }
};

// Chunk LU factors: thread k factorizes rows [s_k, e_k) of A on their own; thread 0 also
// writes the kFactorPad zero rows after row n that the segment kernel reads past the end.
template <int P>
__global__ void part_factor_kernel(const double* __restrict__ A, PartGeom pg, double* __restrict__ F,
                                   double* __restrict__ B)
{
    const int n = pg.n, K = pg.K;
    constexpr int FR = P + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    if (k == 0)
        for (int i = 0; i < kFactorPad * FR; ++i) F[(size_t)n * FR + i] = B[(size_t)n * FR + i] = 0.0;
    lu_rows<P>(A, pg.start(k), pg.start(k + 1), F, B);
}

// Spikes: thread (k, side, j) solves A_kk v = column j of the coupling block (side 0: V_k,
// nonzero right-hand side in the last P rows; side 1: W_k, in the first P rows) into
// rows [s_k, e_k) of V or Wt (P doubles per row).  Spikes that do not exist (V of the last
// chunk, W of the first) are written as zeros.
template <int P>
__global__ void part_spike_kernel(const double* __restrict__ A, PartGeom pg,
                                  const double* __restrict__ F, const double* __restrict__ B,
                                  double* __restrict__ V, double* __restrict__ Wt)
{
    const int K = pg.K;
    constexpr int W = 2 * P + 1, FR = P + 1;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= K * 2 * P) return;
    const int j = id % P, side = (id / P) % 2, k = id / (2 * P);
    const int s = pg.start(k), e = pg.start(k + 1);
    double* out = side == 0 ? V : Wt;
    const bool exists = side == 0 ? k < K - 1 : k > 0;
    double yw[P];
    for (int q = 0; q < P; ++q) yw[q] = 0.0;
    for (int r = s; r < e; ++r) {
        double rhs = 0.0;
        if (exists) {
            const int c = side == 0 ? e + j : s - P + j;
            const bool row_in = side == 0 ? r >= e - P : r < s + P;
            const int kk = c - r + P;
            if (row_in && kk >= 0 && kk <= 2 * P) rhs = A[(size_t)r * W + kk];
        }
        double y = rhs * F[(size_t)r * FR + P];
        for (int q = 0; q < P; ++q) y = fma(-F[(size_t)r * FR + q], yw[q], y);
        out[(size_t)r * P + j] = y;
        for (int q = 0; q + 1 < P; ++q) yw[q] = yw[q + 1];
        yw[P - 1] = y;
    }
    double xw[P];   // xw[q-1] = x_{r+q}
    for (int q = 0; q < P; ++q) xw[q] = 0.0;
    for (int r = e - 1; r >= s; --r) {
        double x = out[(size_t)r * P + j] * B[(size_t)r * FR + P];
        for (int q = P; q >= 1; --q) x = fma(-B[(size_t)r * FR + q - 1], xw[q - 1], x);
        out[(size_t)r * P + j] = x;
        for (int q = P - 1; q >= 1; --q) xw[q] = xw[q - 1];
        xw[0] = x;
    }
}

// In-place inverse of a Q x Q matrix by Gauss-Jordan elimination with partial pivoting.
template <int Q>
__device__ void small_inverse(double (&a)[Q][Q], double (&inv)[Q][Q])
{
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) inv[i][j] = i == j ? 1.0 : 0.0;
    for (int c = 0; c < Q; ++c) {
        int pr = c;
        for (int r = c + 1; r < Q; ++r)
            if (fabs(a[r][c]) > fabs(a[pr][c])) pr = r;
        if (pr != c)
            for (int j = 0; j < Q; ++j) {
                double t = a[c][j];
                a[c][j] = a[pr][j];
                a[pr][j] = t;
                t = inv[c][j];
                inv[c][j] = inv[pr][j];
                inv[pr][j] = t;
            }
        const double d = 1.0 / a[c][c];
        for (int j = 0; j < Q; ++j) {
            a[c][j] *= d;
            inv[c][j] *= d;
        }
        for (int r = 0; r < Q; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            if (f == 0.0) continue;
            for (int j = 0; j < Q; ++j) {
                a[r][j] = fma(-f, a[c][j], a[r][j]);
                inv[r][j] = fma(-f, inv[c][j], inv[r][j]);
            }
        }
    }
}

// Block LU of the reduced system (one thread): Gamma_k (k >= 1; Gamma_0 = 0) and
// Delta_k^{-1} for k = 0 .. K-2, 2P x 2P each, row-major.
template <int P>
__global__ void part_reduce_setup_kernel(const double* __restrict__ V, const double* __restrict__ Wt,
                                         PartGeom pg, double* __restrict__ G, double* __restrict__ Dinv)
{
    const int K = pg.K;
    constexpr int Q = 2 * P;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double prev[Q][Q];   // Delta_{k-1}^{-1}
    for (int k = 0; k + 1 < K; ++k) {
        const int s = pg.start(k), e = pg.start(k + 1);
        double D[Q][Q];
        for (int i = 0; i < Q; ++i)
            for (int j = 0; j < Q; ++j) D[i][j] = i == j ? 1.0 : 0.0;
        for (int i = 0; i < P; ++i)
            for (int j = 0; j < P; ++j) {
                D[i][P + j] = V[(size_t)(e - P + i) * P + j];    // V_k^B
                D[P + i][j] = Wt[(size_t)(e + i) * P + j];       // W_{k+1}^T
            }
        double Gk[Q][Q];
        for (int i = 0; i < Q; ++i)
            for (int j = 0; j < Q; ++j) Gk[i][j] = 0.0;
        if (k >= 1) {
            // Gamma_k = E_k Delta_{k-1}^{-1}: rows 0 .. P-1 are W_k^B times rows 0 .. P-1
            for (int i = 0; i < P; ++i)
                for (int j = 0; j < Q; ++j) {
                    double acc = 0.0;
                    for (int q = 0; q < P; ++q) acc = fma(Wt[(size_t)(e - P + i) * P + q], prev[q][j], acc);
                    Gk[i][j] = acc;
                }
            // Delta_k = D_k - Gamma_k F_{k-1}, F_{k-1} = [0, 0; 0, V_k^T]
            for (int i = 0; i < Q; ++i)
                for (int j = 0; j < P; ++j) {
                    double acc = 0.0;
                    for (int q = 0; q < P; ++q) acc = fma(Gk[i][P + q], V[(size_t)(s + q) * P + j], acc);
                    D[i][P + j] -= acc;
                }
        }
        double inv[Q][Q];
        small_inverse<Q>(D, inv);
        for (int i = 0; i < Q; ++i)
            for (int j = 0; j < Q; ++j) {
                G[((size_t)k * Q + i) * Q + j] = Gk[i][j];
                Dinv[((size_t)k * Q + i) * Q + j] = inv[i][j];
                prev[i][j] = inv[i][j];
            }
    }
}

// Truncated reduced system (the truncated SPIKE scheme of Polizzi and Sameh): the blocks
// E_k and F_k hold the far ends of the spikes, which for chunks of a hundred rows or more
// lie far below rounding; without them the reduced system is block diagonal, and
// zeta_k = D_k^{-1} h_k for every interface at once.  One thread per interface k writes
// D_k^{-1} (row-major) and the largest magnitude of the entries of W_k^B and V_{k+1}^T that
// this drops (NaN if any of them is NaN), from which the host decides.
template <int P>
__global__ __launch_bounds__(64) void part_trunc_setup_kernel(const double* __restrict__ V,
                                                              const double* __restrict__ Wt, PartGeom pg,
                                                              double* __restrict__ Minv, double* __restrict__ tip)
{
    constexpr int Q = 2 * P;
    const int K = pg.K;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K - 1) return;
    const int e = pg.start(k + 1);
    double D[Q][Q], inv[Q][Q];
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) D[i][j] = i == j ? 1.0 : 0.0;
    double m = 0.0;
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            D[i][P + j] = V[(size_t)(e - P + i) * P + j];   // V_k^B
            D[P + i][j] = Wt[(size_t)(e + i) * P + j];      // W_{k+1}^T
            const double w = k >= 1 ? fabs(Wt[(size_t)(e - P + i) * P + j]) : 0.0;     // W_k^B
            const double v = k + 2 < K ? fabs(V[(size_t)(e + i) * P + j]) : 0.0;       // V_{k+1}^T
            if (!(w <= m)) m = w;
            if (!(v <= m)) m = v;
        }
    small_inverse<Q>(D, inv);
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) Minv[((size_t)k * Q + i) * Q + j] = inv[i][j];
    tip[k] = m;
}

// Step 1 for families of fewer lines than a wave has lanes (1D): one thread per
// (line, chunk), lines fastest; a line's row r at (o n + r) inner + i for line
// t = o inner + i.  Rows are read eight at a time ahead of the recurrence.  dst may be src.
template <int P>
__global__ __launch_bounds__(256) void part_local_kernel(const double* __restrict__ F,
                                                         const double* __restrict__ B, PartGeom pg,
                                                         int lines, int inner, const double* src, double* dst)
{
    const int n = pg.n, K = pg.K;
    constexpr int FR = P + 1, U = 8;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= lines * K) return;
    const int t = id % lines, k = id / lines;
    const int o = t / inner, i = t - o * inner;
    const size_t base = (size_t)o * n * inner + i;
    const int s = pg.start(k), e = pg.start(k + 1);
    double yw[P];
#pragma unroll
    for (int q = 0; q < P; ++q) yw[q] = 0.0;
    for (int r0 = s; r0 < e; r0 += U) {
        double bv[U], f[U][FR];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = min(r0 + u, e - 1);
            bv[u] = src[base + (size_t)r * inner];
#pragma unroll
            for (int q = 0; q < FR; ++q) f[u][q] = F[(size_t)r * FR + q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (r0 + u < e) {
                double y = bv[u] * f[u][P];
#pragma unroll
                for (int q = 0; q < P; ++q) y = fma(-f[u][q], yw[q], y);
                dst[base + (size_t)(r0 + u) * inner] = y;
#pragma unroll
                for (int q = 0; q + 1 < P; ++q) yw[q] = yw[q + 1];
                yw[P - 1] = y;
            }
        }
    }
    double xw[P];   // xw[q-1] = x_{r+q}
#pragma unroll
    for (int q = 0; q < P; ++q) xw[q] = 0.0;
    for (int r0 = e - 1; r0 >= s; r0 -= U) {
        double yv[U], bt[U][FR];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = max(r0 - u, s);
            yv[u] = dst[base + (size_t)r * inner];
#pragma unroll
            for (int q = 0; q < FR; ++q) bt[u][q] = B[(size_t)r * FR + q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (r0 - u >= s) {
                double x = yv[u] * bt[u][P];
#pragma unroll
                for (int q = P; q >= 1; --q) x = fma(-bt[u][q - 1], xw[q - 1], x);
                dst[base + (size_t)(r0 - u) * inner] = x;
#pragma unroll
                for (int q = P - 1; q >= 1; --q) xw[q] = xw[q - 1];
                xw[0] = x;
            }
        }
    }
}

// Step 2: one thread per line, T lines per workgroup.  The workgroup first copies the
// block tables (Gamma_k, Delta_k^{-1} and V_{k+1}^T for every k) into LDS, so that the
// sweeps wait on no memory.  Each thread reads all its h_k = x rows e_k - P .. e_k + P - 1
// (k = 0 .. K-2) into LDS, sixteen steps' loads at once (the first sixteen beside the
// table loads), runs the forward sweep there (y_k replaces h_k) and the backward sweep,
// which writes zeta_k to Z (entry (k, q) of line t at Z[(k 2P + q) lines + t]).
// LDS: [tables: (K-1) (2 (2P)^2 + P^2) | T (K-1) 2P].
template <int P>
__host__ __device__ constexpr int part_table_doubles(int K)
{
    return (K - 1) * (2 * 4 * P * P + P * P);
}

template <int P>
__global__ __launch_bounds__(64) void part_reduce_kernel(const double* __restrict__ G,
                                                         const double* __restrict__ Dinv,
                                                         const double* __restrict__ V, PartGeom pg,
                                                         int lines, int inner,
                                                         const double* __restrict__ x, double* __restrict__ Z)
{
    const int n = pg.n, K = pg.K;
    constexpr int Q = 2 * P;
    extern __shared__ double part_y[];
    const int T = blockDim.x, tid = threadIdx.x;
    double* const tabs = part_y;
    const int t = blockIdx.x * T + tid;
    const int tc = min(t, lines - 1);   // lines past the last load the last one's values
    const int o = tc / inner, i = tc - o * inner;
    const size_t base = (size_t)o * n * inner + i;
    constexpr int KB = 16;   // steps whose h is loaded together
    // h of the first KB steps, in flight together with the table loads below
    double hb[KB][Q];
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
        const int e = pg.start(min(kk, K - 2) + 1);
#pragma unroll
        for (int q = 0; q < Q; ++q) hb[kk][q] = x[base + (size_t)(e - P + q) * inner];
    }
    {
        // eight entries per thread in flight at a time: [Gamma | Delta^-1 | V^T]
        const int nq = (K - 1) * Q * Q, nt = 2 * nq + (K - 1) * P * P;
        for (int j0 = 0; j0 < nt; j0 += 8 * T) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = min(j0 + u * T + tid, nt - 1);
                if (j < nq) {
                    v[u] = G[j];
                } else if (j < 2 * nq) {
                    v[u] = Dinv[j - nq];
                } else {
                    const int jj = j - 2 * nq, k = jj / (P * P), a = (jj / P) % P, b = jj % P;
                    v[u] = V[(size_t)(pg.start(k + 1) + a) * P + b];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (j0 + u * T + tid < nt) tabs[j0 + u * T + tid] = v[u];
        }
        __syncthreads();
    }
    if (t >= lines) return;   // no barrier below: each thread uses its own LDS column
    double* yl = part_y + part_table_doubles<P>(K) + tid;
    // block tables in LDS (pointers known to be LDS, so the reads are LDS reads)
    const double* Gp = tabs;
    const double* Dp = tabs + (K - 1) * Q * Q;
    const double* VTs = tabs + 2 * (K - 1) * Q * Q;
    for (int k0 = 0; k0 + 1 < K; k0 += KB) {
        if (k0 > 0) {
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) {
                const int e = pg.start(min(k0 + kk, K - 2) + 1);
#pragma unroll
                for (int q = 0; q < Q; ++q) hb[kk][q] = x[base + (size_t)(e - P + q) * inner];
            }
        }
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
            if (k0 + kk + 1 < K) {
#pragma unroll
                for (int q = 0; q < Q; ++q) yl[(size_t)((k0 + kk) * Q + q) * T] = hb[kk][q];
            }
    }
    // forward: y_k = h_k - Gamma_k y_{k-1}
    double y[Q], g[Q * Q], gn[Q * Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) y[q] = yl[(size_t)q * T];
#pragma unroll
    for (int q = 0; q < Q * Q; ++q) gn[q] = K > 2 ? Gp[(size_t)Q * Q + q] : 0.0;
    for (int k = 1; k + 1 < K; ++k) {
#pragma unroll
        for (int q = 0; q < Q * Q; ++q) g[q] = gn[q];
        const int kn = k + 2 < K ? k + 1 : k;
#pragma unroll
        for (int q = 0; q < Q * Q; ++q) gn[q] = Gp[(size_t)kn * Q * Q + q];
        double h[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            double acc = yl[(size_t)(k * Q + a) * T];
#pragma unroll
            for (int b = 0; b < Q; ++b) acc = fma(-g[a * Q + b], y[b], acc);
            h[a] = acc;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            y[q] = h[q];
            yl[(size_t)(k * Q + q) * T] = h[q];
        }
    }
    // backward: zeta_k = Delta_k^{-1} (y_k - F_k zeta_{k+1})
    double zn[Q], d[Q * Q], dn[Q * Q], vt[P * P], vn[P * P];
#pragma unroll
    for (int q = 0; q < Q * Q; ++q) dn[q] = Dp[(size_t)(K - 2) * Q * Q + q];
#pragma unroll
    for (int q = 0; q < P * P; ++q) vn[q] = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) zn[q] = 0.0;
    for (int k = K - 2; k >= 0; --k) {
#pragma unroll
        for (int q = 0; q < Q * Q; ++q) d[q] = dn[q];
#pragma unroll
        for (int q = 0; q < P * P; ++q) vt[q] = vn[q];   // V_{k+1}^T (0 for k = K-2)
        const int kn = k > 0 ? k - 1 : k;
#pragma unroll
        for (int q = 0; q < Q * Q; ++q) dn[q] = Dp[(size_t)kn * Q * Q + q];
#pragma unroll
        for (int q = 0; q < P * P; ++q) vn[q] = VTs[(size_t)kn * P * P + q];
        double rhs[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) rhs[q] = yl[(size_t)(k * Q + q) * T];
#pragma unroll
        for (int a = 0; a < P; ++a) {
            double acc = rhs[P + a];
#pragma unroll
            for (int b = 0; b < P; ++b) acc = fma(-vt[a * P + b], zn[P + b], acc);
            rhs[P + a] = acc;
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < Q; ++b) acc = fma(d[a * Q + b], rhs[b], acc);
            zn[a] = acc;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) Z[((size_t)k * Q + q) * lines + t] = zn[q];
    }
}

// Step 2 for long chains (block tables too large for LDS; a single long line): the
// workgroup's 64 threads stream the tables through an LDS ring, kStreamSteps steps at a
// time, the next batch loading while the first TL threads (one line each) run the
// current one.  LDS: [ring: 2 kStreamSteps (2P)^2 + P^2 | TL (K-1) 2P].
constexpr int kStreamSteps = 16;
template <int P>
__host__ __device__ constexpr int part_stream_ring_doubles()
{
    return 2 * kStreamSteps * (4 * P * P + P * P);
}

template <int P>
__global__ __launch_bounds__(64) void part_reduce_stream_kernel(const double* __restrict__ G,
                                                                const double* __restrict__ Dinv,
                                                                const double* __restrict__ V, PartGeom pg,
                                                                int lines, int inner, int TL,
                                                                const double* __restrict__ x,
                                                                double* __restrict__ Z)
{
    constexpr int Q = 2 * P, QQ = Q * Q, PP = P * P, EW = QQ + PP;   // ring entry: Q^2 (+ P^2)
    constexpr int SH = (kStreamSteps * EW + 63) / 64;                // ring doubles per thread
    const int n = pg.n, K = pg.K;
    constexpr int kSweepUnroll = P == 2 ? 4 : 1;   // p = 3 needs the registers
    extern __shared__ double part_y[];
    double* const ring = part_y;                                     // 2 halves of kStreamSteps EW
    const int tid = threadIdx.x;
    const int t = blockIdx.x * TL + tid;
    const bool active = tid < TL && t < lines;
    const int tc = min(active ? t : blockIdx.x * TL, lines - 1);
    const int o = tc / inner, i = tc - o * inner;
    const size_t base = (size_t)o * n * inner + i;
    double* yl = part_y + part_stream_ring_doubles<P>() + tid;
    const int nst = K - 1;   // steps 0 .. K-2
    if (active)
        for (int k0 = 0; k0 < nst; k0 += kStreamSteps) {   // a batch of steps' loads at once
            double hb[kStreamSteps][Q];
#pragma unroll
            for (int kk = 0; kk < kStreamSteps; ++kk) {
                const int e = pg.start(min(k0 + kk, nst - 1) + 1);
#pragma unroll
                for (int q = 0; q < Q; ++q) hb[kk][q] = x[base + (size_t)(e - P + q) * inner];
            }
#pragma unroll
            for (int kk = 0; kk < kStreamSteps; ++kk)
                if (k0 + kk < nst) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) yl[(size_t)((k0 + kk) * Q + q) * TL] = hb[kk][q];
                }
        }
    // one batch of ring entries: forward entries hold Gamma_k; backward entries Delta_k^{-1}
    // and V_{k+1}^T (step k of the batch order; its entry at e * EW)
    auto fetch = [&](bool fwd, int b, double (&reg)[SH]) {
#pragma unroll
        for (int u = 0; u < SH; ++u) {
            const int j = u * 64 + tid;
            const int e = j / EW, w = j - e * EW;
            const int kk = fwd ? 1 + b * kStreamSteps + e : nst - 1 - (b * kStreamSteps + e);
            double v = 0.0;
            if (j < kStreamSteps * EW && kk >= 0 && kk < nst) {
                if (w < QQ)
                    v = fwd ? G[(size_t)kk * QQ + w] : Dinv[(size_t)kk * QQ + w];
                else if (!fwd && kk + 1 < nst)
                    v = V[(size_t)(pg.start(kk + 1) + (w - QQ) / P) * P + (w - QQ) % P];
            }
            reg[u] = v;
        }
    };
    auto put = [&](int half, const double (&reg)[SH]) {
#pragma unroll
        for (int u = 0; u < SH; ++u) {
            const int j = u * 64 + tid;
            if (j < kStreamSteps * EW) ring[half * kStreamSteps * EW + j] = reg[u];
        }
    };
    double reg[SH];
    // forward: y_k = h_k - Gamma_k y_{k-1}, k = 1 .. K-2 in batches
    double y[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) y[q] = active ? yl[(size_t)q * TL] : 0.0;
    const int nbf = (nst - 1 + kStreamSteps - 1) / kStreamSteps;
    fetch(true, 0, reg);
    put(0, reg);
    __syncthreads();
    for (int b = 0; b < nbf; ++b) {
        fetch(true, b + 1, reg);
        if (active) {
            const double* rb = ring + (b & 1) * kStreamSteps * EW;
            const int ne = min(kStreamSteps, nst - 1 - b * kStreamSteps);   // steps of this batch
#pragma unroll(kSweepUnroll)
            for (int e = 0; e < ne; ++e) {
                const int k = 1 + b * kStreamSteps + e;
                double h[Q];
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    double acc = yl[(size_t)(k * Q + a) * TL];
#pragma unroll
                    for (int c = 0; c < Q; ++c) acc = fma(-rb[e * EW + a * Q + c], y[c], acc);
                    h[a] = acc;
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    y[q] = h[q];
                    yl[(size_t)(k * Q + q) * TL] = h[q];
                }
            }
        }
        put((b + 1) & 1, reg);
        __syncthreads();
    }
    // backward: zeta_k = Delta_k^{-1} (y_k - F_k zeta_{k+1}), k = K-2 .. 0 in batches
    double zn[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) zn[q] = 0.0;
    const int nbb = (nst + kStreamSteps - 1) / kStreamSteps;
    fetch(false, 0, reg);
    put(0, reg);
    __syncthreads();
    for (int b = 0; b < nbb; ++b) {
        fetch(false, b + 1, reg);
        if (active) {
            const double* rb = ring + (b & 1) * kStreamSteps * EW;
            const int ne = min(kStreamSteps, nst - b * kStreamSteps);   // steps of this batch
#pragma unroll(kSweepUnroll)
            for (int e = 0; e < ne; ++e) {
                const int k = nst - 1 - (b * kStreamSteps + e);
                // the entry of step k holds Delta_k^{-1} and V_{k+1}^T
                double rhs[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) rhs[q] = yl[(size_t)(k * Q + q) * TL];
                if (k < nst - 1) {
                    const double* vt = rb + e * EW + QQ;
#pragma unroll
                    for (int a = 0; a < P; ++a) {
                        double acc = rhs[P + a];
#pragma unroll
                        for (int c = 0; c < P; ++c) acc = fma(-vt[a * P + c], zn[P + c], acc);
                        rhs[P + a] = acc;
                    }
                }
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    double acc = 0.0;
#pragma unroll
                    for (int c = 0; c < Q; ++c) acc = fma(rb[e * EW + a * Q + c], rhs[c], acc);
                    zn[a] = acc;
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) Z[((size_t)k * Q + q) * lines + t] = zn[q];
            }
        }
        put((b + 1) & 1, reg);
        __syncthreads();
    }
}

// Step 3: x -= V[r] t_{k+1} + Wt[r] u_{k-1} on every value, kCorr values per thread with
// every load issued before the first is used.  A single line: 256 threads per workgroup
// flat over its rows (one chunk lookup per row; a workgroup per chunk leaves 10^4 small
// workgroups for a line of 10^6 rows in chunks of 96).  x-lines (inner = 1): a workgroup
// per (chunk, kCorr lines) = (blockIdx.x, blockIdx.y), its threads over the chunk's rows.
// Other families: a workgroup per (kCorr rows of line groups, inner block) =
// (blockIdx.x, blockIdx.y), its threads over the inner index.  The chunk of a row is
// uniform across the workgroup, so no thread divides.
constexpr int kCorr = 4;
template <int P>
__global__ __launch_bounds__(256) void part_correct_kernel(const double* __restrict__ V,
                                                           const double* __restrict__ Wt, PartGeom pg,
                                                           int lines, int inner, int rows,
                                                           const double* __restrict__ Z, double* __restrict__ x)
{
    const int n = pg.n, K = pg.K;
    constexpr int Q = 2 * P;
    if (lines == 1) {
        // a single line (inner = 1): flat over its rows, kCorr rows per thread a workgroup
        // apart; interior chunks of equal length (m > 0) have bitwise equal spikes, and all
        // read chunk 1's, which stay in the cache
        double xv[kCorr], vr[kCorr][P], wr[kCorr][P], zt[kCorr][P], zu[kCorr][P];
        const int rb = blockIdx.x * blockDim.x * kCorr + threadIdx.x;
#pragma unroll
        for (int u = 0; u < kCorr; ++u) {
            const int r = min(rb + u * (int)blockDim.x, n - 1);
            const int k = pg.chunk(r);
            const int rs = pg.m > 0 && k > 0 && k + 1 < K ? r - pg.start(k) + pg.start(1) : r;
            xv[u] = x[r];
#pragma unroll
            for (int j = 0; j < P; ++j) {
                vr[u][j] = V[(size_t)rs * P + j];
                wr[u][j] = Wt[(size_t)rs * P + j];
                zt[u][j] = k < K - 1 ? Z[(size_t)k * Q + P + j] : 0.0;
                zu[u][j] = k > 0 ? Z[(size_t)(k - 1) * Q + j] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < kCorr; ++u) {
            double v = xv[u];
#pragma unroll
            for (int j = 0; j < P; ++j) v = fma(-vr[u][j], zt[u][j], v);
#pragma unroll
            for (int j = 0; j < P; ++j) v = fma(-wr[u][j], zu[u][j], v);
            if (rb + u * (int)blockDim.x < n) x[rb + u * blockDim.x] = v;
        }
        return;
    }
    if (inner == 1) {
        const int k = blockIdx.x, o0 = blockIdx.y * kCorr;
        const int r1 = pg.start(k + 1);
        double zt[kCorr][P], zu[kCorr][P];
#pragma unroll
        for (int u = 0; u < kCorr; ++u) {
            const int o = min(o0 + u, lines - 1);
#pragma unroll
            for (int j = 0; j < P; ++j) {
                zt[u][j] = k < K - 1 ? Z[((size_t)k * Q + P + j) * lines + o] : 0.0;
                zu[u][j] = k > 0 ? Z[((size_t)(k - 1) * Q + j) * lines + o] : 0.0;
            }
        }
        for (int r = pg.start(k) + threadIdx.x; r < r1; r += blockDim.x) {
            double vr[P], wr[P], xv[kCorr];
#pragma unroll
            for (int j = 0; j < P; ++j) {
                vr[j] = V[(size_t)r * P + j];
                wr[j] = Wt[(size_t)r * P + j];
            }
#pragma unroll
            for (int u = 0; u < kCorr; ++u) xv[u] = x[(size_t)min(o0 + u, lines - 1) * n + r];
#pragma unroll
            for (int u = 0; u < kCorr; ++u) {
                double v = xv[u];
#pragma unroll
                for (int j = 0; j < P; ++j) v = fma(-vr[j], zt[u][j], v);
#pragma unroll
                for (int j = 0; j < P; ++j) v = fma(-wr[j], zu[u][j], v);
                if (o0 + u < lines) x[(size_t)(o0 + u) * n + r] = v;
            }
        }
        return;
    }
    const int i = blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= inner) return;
    double xv[kCorr], zt[kCorr][P], zu[kCorr][P], vr[kCorr][P], wr[kCorr][P];
    size_t idx[kCorr];
#pragma unroll
    for (int u = 0; u < kCorr; ++u) {
        const int g = min(blockIdx.x * kCorr + u, rows - 1), o = g / n, r = g - o * n;
        const int k = pg.chunk(r);
        const int t = o * inner + i;
        idx[u] = ((size_t)o * n + r) * inner + i;
        xv[u] = x[idx[u]];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            zt[u][j] = k < K - 1 ? Z[((size_t)k * Q + P + j) * lines + t] : 0.0;
            zu[u][j] = k > 0 ? Z[((size_t)(k - 1) * Q + j) * lines + t] : 0.0;
            vr[u][j] = V[(size_t)r * P + j];
            wr[u][j] = Wt[(size_t)r * P + j];
        }
    }
#pragma unroll
    for (int u = 0; u < kCorr; ++u) {
        double v = xv[u];
#pragma unroll
        for (int j = 0; j < P; ++j) v = fma(-vr[u][j], zt[u][j], v);
#pragma unroll
        for (int j = 0; j < P; ++j) v = fma(-wr[u][j], zu[u][j], v);
        if (blockIdx.x * kCorr + u < (unsigned)rows) x[idx[u]] = v;
    }
}

// Steps 2 and 3 of the block-diagonal reduced system in one launch, out of place: the
// chunk solves left g in w, which nothing here writes, so each workgroup first solves the
// interfaces its rows need, zeta_k = D_k^{-1} h_k with h_k read from w, and then writes
// x = g - V_k t_{k+1} - W_k u_{k-1}.  The mappings are those of part_correct_kernel.  A
// single line's workgroup spans 1024 rows; its chunks have at least 63 rows but for two
// end chunks of at least 16, so it needs at most 21 interfaces (kFixIf bounds the LDS).
// With ends set (a single line in equal interior chunks, m > 0), the end chunks were not
// solved beforehand: a workgroup whose rows reach chunk 0 or 1 (K-2 or K-1) solves chunk 0
// (K-1) itself from src, staged in LDS, one thread running the two substitutions, and
// takes that chunk's g from LDS (at most kFixEnd rows; the two workgroups at a chunk
// boundary both solve it).
constexpr int kFixIf = 32;
constexpr int kFixEnd = 80;
template <int P>
__global__ __launch_bounds__(256) void part_fix_kernel(const double* __restrict__ V,
                                                       const double* __restrict__ Wt,
                                                       const double* __restrict__ Minv, PartGeom pg,
                                                       int lines, int inner, int rows,
                                                       const double* __restrict__ w, double* __restrict__ x,
                                                       const double* __restrict__ F, const double* __restrict__ B,
                                                       const double* __restrict__ src, int ends)
{
    const int n = pg.n, K = pg.K;
    constexpr int Q = 2 * P, FR = P + 1;
    __shared__ double zl[kFixIf * Q];
    __shared__ double el[2][kFixEnd];          // g of the first / last chunk
    __shared__ double et[kFixEnd * 2 * FR];    // their factor rows while one is solved
    int e0 = -1, e1 = n;                       // rows below e0 / from e1 on come from el
    // g of row r of the line at base
    auto gval = [&](size_t base, int r) -> double {
        if (r < e0) return el[0][r];
        if (r >= e1) return el[1][r - e1];
        return w[base + (size_t)r * inner];
    };
    // entries a0 .. a0+na-1 of zeta_kk of the line whose row r is at base + r inner
    auto solve_if = [&](int kk, size_t base, int a0, int na, double* z) {
        const int e = pg.start(kk + 1);
        double h[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) h[q] = gval(base, e - P + q);
        const double* M = Minv + (size_t)kk * Q * Q;
        for (int a = 0; a < na; ++a) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < Q; ++c) acc = fma(M[(a0 + a) * Q + c], h[c], acc);
            z[a] = acc;
        }
    };
    double gv[kCorr], vr[kCorr][P], wr[kCorr][P], zt[kCorr][P], zu[kCorr][P];
    if (lines == 1) {
        const int r0 = blockIdx.x * blockDim.x * kCorr;
        const int ka = pg.chunk(r0), kb = pg.chunk(min(r0 + (int)blockDim.x * kCorr - 1, n - 1));
        if (ends)
            for (int side = 0; side < 2; ++side) {   // uniform across the workgroup
                if (side == 0 ? ka > 1 : kb < K - 2) continue;
                const int s0 = side == 0 ? 0 : pg.start(K - 1), len = min(side == 0 ? pg.start(1) : n - s0, kFixEnd);
                for (int t = threadIdx.x; t < len; t += blockDim.x) {
                    el[side][t] = src[s0 + t];
#pragma unroll
                    for (int q = 0; q < FR; ++q) {
                        et[t * 2 * FR + q] = F[(size_t)(s0 + t) * FR + q];
                        et[t * 2 * FR + FR + q] = B[(size_t)(s0 + t) * FR + q];
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) {   // forward y_r = b_r F_rP - sum F_rq y_{r-P+q}, then backward
                    double yw[P];
#pragma unroll
                    for (int q = 0; q < P; ++q) yw[q] = 0.0;
                    for (int t = 0; t < len; ++t) {
                        double y = el[side][t] * et[t * 2 * FR + P];
#pragma unroll
                        for (int q = 0; q < P; ++q) y = fma(-et[t * 2 * FR + q], yw[q], y);
                        el[side][t] = y;
#pragma unroll
                        for (int q = 0; q + 1 < P; ++q) yw[q] = yw[q + 1];
                        yw[P - 1] = y;
                    }
                    double xw[P];   // xw[q-1] = x_{t+q}
#pragma unroll
                    for (int q = 0; q < P; ++q) xw[q] = 0.0;
                    for (int t = len - 1; t >= 0; --t) {
                        double v = el[side][t] * et[t * 2 * FR + FR + P];
#pragma unroll
                        for (int q = P; q >= 1; --q) v = fma(-et[t * 2 * FR + FR + q - 1], xw[q - 1], v);
                        el[side][t] = v;
#pragma unroll
                        for (int q = P - 1; q >= 1; --q) xw[q] = xw[q - 1];
                        xw[0] = v;
                    }
                }
                __syncthreads();
                if (side == 0) e0 = len;
                else e1 = s0;
            }
        const int nif = min(kb - ka + 2, kFixIf);   // interfaces ka-1 .. kb
        for (int t = threadIdx.x; t < nif; t += blockDim.x) {
            const int kk = ka - 1 + t;
            if (kk >= 0 && kk <= K - 2) solve_if(kk, 0, 0, Q, zl + t * Q);
        }
        __syncthreads();
        const int rb = r0 + threadIdx.x;
#pragma unroll
        for (int u = 0; u < kCorr; ++u) {
            const int r = min(rb + u * (int)blockDim.x, n - 1);
            const int k = pg.chunk(r);
            const int rs = pg.m > 0 && k > 0 && k + 1 < K ? r - pg.start(k) + pg.start(1) : r;
            const int it = min(k - ka + 1, kFixIf - 1), iu = min(k - ka, kFixIf - 1);
            gv[u] = gval(0, r);
#pragma unroll
            for (int j = 0; j < P; ++j) {
                vr[u][j] = V[(size_t)rs * P + j];
                wr[u][j] = Wt[(size_t)rs * P + j];
                zt[u][j] = k < K - 1 ? zl[it * Q + P + j] : 0.0;
                zu[u][j] = k > 0 ? zl[iu * Q + j] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < kCorr; ++u) {
            double v = gv[u];
#pragma unroll
            for (int j = 0; j < P; ++j) v = fma(-vr[u][j], zt[u][j], v);
#pragma unroll
            for (int j = 0; j < P; ++j) v = fma(-wr[u][j], zu[u][j], v);
            if (rb + u * (int)blockDim.x < n) x[rb + u * blockDim.x] = v;
        }
        return;
    }
    if (inner == 1) {
        // threads 2u + s solve zeta_{k-1+s} of line o0 + u into LDS
        const int k = blockIdx.x, o0 = blockIdx.y * kCorr;
        if (threadIdx.x < 2 * kCorr) {
            const int u = threadIdx.x >> 1, kk = k - 1 + (threadIdx.x & 1);
            if (kk >= 0 && kk <= K - 2) solve_if(kk, (size_t)min(o0 + u, lines - 1) * n, 0, Q, zl + threadIdx.x * Q);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kCorr; ++u)
#pragma unroll
            for (int j = 0; j < P; ++j) {
                zt[u][j] = k < K - 1 ? zl[(2 * u + 1) * Q + P + j] : 0.0;
                zu[u][j] = k > 0 ? zl[2 * u * Q + j] : 0.0;
            }
        const int r1 = pg.start(k + 1);
        for (int r = pg.start(k) + threadIdx.x; r < r1; r += blockDim.x) {
            double vk[P], wk[P];
#pragma unroll
            for (int j = 0; j < P; ++j) {
                vk[j] = V[(size_t)r * P + j];
                wk[j] = Wt[(size_t)r * P + j];
            }
#pragma unroll
            for (int u = 0; u < kCorr; ++u) gv[u] = w[(size_t)min(o0 + u, lines - 1) * n + r];
#pragma unroll
            for (int u = 0; u < kCorr; ++u) {
                double v = gv[u];
#pragma unroll
                for (int j = 0; j < P; ++j) v = fma(-vk[j], zt[u][j], v);
#pragma unroll
                for (int j = 0; j < P; ++j) v = fma(-wk[j], zu[u][j], v);
                if (o0 + u < lines) x[(size_t)(o0 + u) * n + r] = v;
            }
        }
        return;
    }
    // other families: the rows of a workgroup are uniform across it, and so is the change
    // of (line group, chunk) from one row to the next, where the thread solves anew
    const int i = blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= inner) return;
    size_t idx[kCorr];
    int po = -1, pk = -1;
    double ct[P], cu[P];
#pragma unroll
    for (int u = 0; u < kCorr; ++u) {
        const int g = min(blockIdx.x * kCorr + u, rows - 1), o = g / n, r = g - o * n;
        const int k = pg.chunk(r);
        const size_t base = (size_t)o * n * inner + i;
        if (o != po || k != pk) {
            if (k < K - 1) solve_if(k, base, P, P, ct);
            else
                for (int j = 0; j < P; ++j) ct[j] = 0.0;
            if (k > 0) solve_if(k - 1, base, 0, P, cu);
            else
                for (int j = 0; j < P; ++j) cu[j] = 0.0;
            po = o;
            pk = k;
        }
        idx[u] = base + (size_t)r * inner;
        gv[u] = w[idx[u]];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            zt[u][j] = ct[j];
            zu[u][j] = cu[j];
            vr[u][j] = V[(size_t)r * P + j];
            wr[u][j] = Wt[(size_t)r * P + j];
        }
    }
#pragma unroll
    for (int u = 0; u < kCorr; ++u) {
        double v = gv[u];
#pragma unroll
        for (int j = 0; j < P; ++j) v = fma(-vr[u][j], zt[u][j], v);
#pragma unroll
        for (int j = 0; j < P; ++j) v = fma(-wr[u][j], zu[u][j], v);
        if (blockIdx.x * kCorr + u < (unsigned)rows) x[idx[u]] = v;
    }
}

}  // namespace iga
