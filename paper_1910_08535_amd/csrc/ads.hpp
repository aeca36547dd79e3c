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

typedef int iv2s __attribute__((ext_vector_type(2)));
typedef int iv4s __attribute__((ext_vector_type(4)));
typedef double dv2s __attribute__((ext_vector_type(2)));

// Factor tables of one axis, P+1 doubles per row, kFactorPad rows of zeros after the
// last row (rows past the end of a line then solve to 0 and couple to nothing, so the
// substitutions need no bounds tests; kFactorPad covers the padding of the last segment
// plus the band):
//   L: [L(r, r-P), ..., L(r, r-1), 1 / L(r, r)]        (entries of columns < 0 are 0)
//   F: [L(r, r-P) d_r, ..., L(r, r-1) d_r, d_r]         d_r = 1 / L(r, r)
//   B: [L(r+1, r) d_r, ..., L(r+P, r) d_r, d_r]
// With F and B the forward step is y_r = b_r d_r - sum_k F(r,k) y_{r-P+k} and the backward
// step x_r = y_r d_r - sum_j B(r,j-1) x_{r+j}: the newest value enters one FMA only.
constexpr int kFactorPad = 128;

// Banded LU without pivoting of rows r0 .. r1-1 of a banded matrix A (rows of 2P+1
// doubles, A[r (2P+1) + c - r + P] = A(r, c)) taken on its own: columns outside [r0, r1)
// are dropped.  A = L U with L unit lower and U upper, both of bandwidth P; rows r0 .. r1-1
// of the sweep tables get F[r] = [L(r, r-P), ..., L(r, r-1), 1] and
// B[r] = [U(r, r+1) d_r, ..., U(r, r+P) d_r, d_r], d_r = 1 / U(r, r) (entries of columns
// outside the range 0), so the substitutions are those of the Cholesky tables.  One thread.
template <int P>
__device__ void lu_rows(const double* __restrict__ A, int r0, int r1, double* __restrict__ F,
                        double* __restrict__ B)
{
    constexpr int W = 2 * P + 1, FR = P + 1;
    double ur[P][P + 1];   // rows r-P .. r-1 of U: ur[j][k] = U(r-P+j, r-P+j+k)
    for (int j = 0; j < P; ++j)
        for (int k = 0; k <= P; ++k) ur[j][k] = 0.0;
    for (int r = r0; r < r1; ++r) {
        const double* ar = A + (size_t)r * W;   // ar[c - r + P] = A(r, c)
        double l[P];
        for (int k = 0; k < P; ++k) {           // column c = r - P + k < r
            const int c = r - P + k;
            if (c < r0) {
                l[k] = 0.0;
                continue;
            }
            double s = ar[k];
            for (int m = 0; m < k; ++m) {       // rows r - P + m < c with U(., c) in band
                const int row = r - P + m;
                if (row < r0 || c - row > P) continue;
                s = fma(-l[m], ur[m][c - row], s);
            }
            l[k] = s / ur[k][0];
        }
        double u[P + 1];
        for (int k = 0; k <= P; ++k) {          // column c = r + k
            const int c = r + k;
            double s = ar[P + k];
            for (int m = 0; m < P; ++m) {
                const int row = r - P + m;
                if (row < r0 || c - row > P) continue;
                s = fma(-l[m], ur[m][c - row], s);
            }
            u[k] = c < r1 ? s : 0.0;
        }
        const double d = 1.0 / u[0];
        for (int k = 0; k < P; ++k) F[(size_t)r * FR + k] = l[k];
        F[(size_t)r * FR + P] = 1.0;
        for (int j = 1; j <= P; ++j) B[(size_t)r * FR + j - 1] = u[j] * d;
        B[(size_t)r * FR + P] = d;
        for (int j = 0; j + 1 < P; ++j)
            for (int k = 0; k <= P; ++k) ur[j][k] = ur[j + 1][k];
        for (int k = 0; k <= P; ++k) ur[P - 1][k] = u[k];
    }
}

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
    for (int i = threadIdx.x; i < kFactorPad * FR; i += blockDim.x) L[(size_t)N * FR + i] = 0.0;
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

// Lane l's value of v (a register move to a scalar register; l is a constant).
__device__ __forceinline__ double lane_value(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// F and B from L, one thread per row (pad rows included).
template <int P>
__global__ void scaled_factor_kernel(const double* __restrict__ L, int N, double* __restrict__ F,
                                     double* __restrict__ B)
{
    constexpr int FR = P + 1;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N + kFactorPad) return;
    if (r >= N) {
#pragma unroll
        for (int k = 0; k < FR; ++k) F[(size_t)r * FR + k] = B[(size_t)r * FR + k] = 0.0;
        return;
    }
    const double d = L[(size_t)r * FR + P];
#pragma unroll
    for (int k = 0; k < P; ++k) F[(size_t)r * FR + k] = L[(size_t)r * FR + k] * d;
#pragma unroll
    for (int j = 1; j <= P; ++j) B[(size_t)r * FR + j - 1] = L[(size_t)(r + j) * FR + P - j] * d;
    F[(size_t)r * FR + P] = d;
    B[(size_t)r * FR + P] = d;
}

// ---------------------------------------------------------------------------------
// One family of 1D solves: x = (L L^T)^{-1} b along every line of one axis.
// Line t = (o, i), o in [0, lines / inner), i in [0, inner): element r (0 <= r < n) of
// the line sits at o * n * inner + r * inner + i.  So inner = 1 walks x-lines (rows of
// the array), inner = N_x walks y-lines and inner = N_x N_y walks z-lines; consecutive
// threads take consecutive i, which makes the y and z families' accesses coalesced.
// One thread per line (one wave per workgroup): the forward substitution writes y over
// x, the backward one reads it back in reverse.  Each direction keeps the next U = 64
// values of its line in flight (double-buffered), and the factor rows of those 64 rows
// one per lane (read with register moves), so that the recurrence waits on memory once
// per 64 rows: this path serves lines too long to stay on chip, and there are few of
// them.  Lanes past the last line repeat it and store nothing.
// x may equal b.  L rows are uniform across a wave (scalar loads).
// ---------------------------------------------------------------------------------
constexpr int kAdsBlock = 64;   // few lines take this path: one wave per CU

template <int P>
__global__ __launch_bounds__(kAdsBlock) void ads_sweep_kernel(const double* __restrict__ F,
                                                              const double* __restrict__ B, int n,
                                                              long long lines, long long inner,
                                                              const double* b, double* x)
{
    constexpr int FR = P + 1, U = 64;
    static_assert(U == 64, "lane u holds the factor row of step u of a block");
    const int lane = threadIdx.x;
    const long long t = (long long)blockIdx.x * kAdsBlock + lane;
    const bool live = t < lines;
    const long long tl = live ? t : lines - 1;
    const long long o = tl / inner, i = tl - o * inner;
    const double* bl = b + o * (long long)n * inner + i;
    double* xl = x + o * (long long)n * inner + i;

    // forward: y_r = b_r d_r - sum_k F(r, k) y_{r-P+k}
    double yw[P];
#pragma unroll
    for (int k = 0; k < P; ++k) yw[k] = 0.0;
    double cur[U], nxt[U], fc[FR], fn[FR];
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = bl[(long long)min(u, n - 1) * inner];
#pragma unroll
    for (int k = 0; k < FR; ++k) fc[k] = F[(size_t)min(lane, n - 1) * FR + k];
    for (int r0 = 0; r0 < n; r0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = bl[(long long)min(r0 + U + u, n - 1) * inner];
#pragma unroll
        for (int k = 0; k < FR; ++k) fn[k] = F[(size_t)min(r0 + U + lane, n - 1) * FR + k];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 + u;
            if (r < n) {
                double f[FR];
#pragma unroll
                for (int k = 0; k < FR; ++k) f[k] = lane_value(fc[k], u);
                double y = cur[u] * f[P];
#pragma unroll
                for (int k = 0; k < P; ++k) y = fma(-f[k], yw[k], y);
                if (live) xl[(long long)r * inner] = y;
#pragma unroll
                for (int k = 0; k + 1 < P; ++k) yw[k] = yw[k + 1];
                yw[P - 1] = y;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
#pragma unroll
        for (int k = 0; k < FR; ++k) fc[k] = fn[k];
    }

    // backward: x_r = y_r d_r - sum_{k=1..P} B(r, k-1) x_{r+k}; the zero rows after the
    // table make the terms beyond the line vanish
    double xw[P];   // xw[k-1] = x_{r+k}
#pragma unroll
    for (int k = 0; k < P; ++k) xw[k] = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = xl[(long long)max(n - 1 - u, 0) * inner];
#pragma unroll
    for (int k = 0; k < FR; ++k) fc[k] = B[(size_t)max(n - 1 - lane, 0) * FR + k];
    for (int r0 = n - 1; r0 >= 0; r0 -= U) {
#pragma unroll
        for (int u = 0; u < U; ++u) nxt[u] = xl[(long long)max(r0 - U - u, 0) * inner];
#pragma unroll
        for (int k = 0; k < FR; ++k) fn[k] = B[(size_t)max(r0 - U - lane, 0) * FR + k];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 - u;
            if (r >= 0) {
                double f[FR];
#pragma unroll
                for (int k = 0; k < FR; ++k) f[k] = lane_value(fc[k], u);
                double v = cur[u] * f[P];
#pragma unroll
                for (int k = P; k >= 1; --k) v = fma(-f[k - 1], xw[k - 1], v);
                if (live) xl[(long long)r * inner] = v;
#pragma unroll
                for (int k = P - 1; k >= 1; --k) xw[k] = xw[k - 1];
                xw[0] = v;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
#pragma unroll
        for (int k = 0; k < FR; ++k) fc[k] = fn[k];
    }
}

// ---------------------------------------------------------------------------------
// The same family of solves with every line held on chip, for lines of at most
// kSegMaxWaves * kSeg rows.  A workgroup owns 64 consecutive lines (one per lane); its
// wave w holds rows [w * kSeg, (w+1) * kSeg) of them in registers, all loaded at once at
// the start, so memory sees one read and one write per value.  The recurrences then run
// wave after wave: forward from wave 0 up, each wave handing the last P values of its
// lines to the next through LDS, backward from the last wave down, each wave handing its
// first P values down and storing its rows.  Lanes past the last line repeat the last
// line and store nothing.  With HALVES = 2 (lines of up to twice as many rows) a wave
// holds two halves of 32 lines: lanes 0-31 rows [w kSeg, ...) of the first half of the
// lines, lanes 32-63 rows [(nw + w) kSeg, ...) of the second; the recurrences then run
// over 2 nw phases, and the factor rows held in lanes are reloaded for the other half.
// Addressing: a buffer resource based at the wave's first element, one 32-bit lane
// offset, and the row stride in the scalar offset, so that no per-row address is kept
// (the host checks that every offset fits 32 bits).  The factor rows of a wave's kSeg
// rows are loaded with the values, lane s holding row r0 + s, and each step of the
// recurrences takes its row from lane s with a register read: no memory latency per row.
//
// x-lines (CONTIG) are contiguous, so a lane's rows lie one line length away from the
// next lane's and lane-per-line accesses touch 64 cache lines per instruction.  Their
// values instead pass through a per-wave LDS stage, kStageRows rows of the wave's 64
// segments at a time: the loads go straight into LDS (buffer loads with the LDS flag),
// eight lanes covering the 128 contiguous bytes of one segment, and each lane then reads
// its own rows back; the stores take the reverse route.
// ---------------------------------------------------------------------------------
constexpr int kSeg = 48;   // even: the contiguous variant moves rows in pairs
constexpr int kSegMaxWaves = 16;
constexpr int kStageRows = 16;                     // rows of a segment per stage pass
constexpr int kStageBytes = 64 * kStageRows * 8;   // stage of one wave
static_assert(kSeg % kStageRows == 0 && kStageRows == 16, "a stage pass moves 8 pairs per segment");
static_assert(kFactorPad >= 2 * kSeg + 3, "zero rows must cover the padding of two halves and the band");

__device__ __forceinline__ unsigned opaque_val(unsigned v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// Orders the LDS accesses of one wave around it (the wave's LDS operations execute in
// order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Waits for every outstanding vector memory operation (s_waitcnt vmcnt(0)): loads into
// LDS are not tracked by the compiler's waits.
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// Waits for every outstanding LDS operation (s_waitcnt lgkmcnt(0)).
__device__ __forceinline__ void wait_lds_all() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Byte position in a wave's stage of pair 0 (rows 0, 1 of the pass) of segment L; pair j
// sits at stage_pos(L) ^ 16 j.  Transfer instruction q moves segments 8q .. 8q+7, its lane
// 8a + b pair b ^ a of segment 8q + a, to bytes 16 (64 q + lane): contiguous for the loads
// into LDS, and the XOR puts the eight segments a lane group reads back at one pair index
// in distinct banks.
__device__ __forceinline__ unsigned stage_pos(int L)
{
    const int a = L & 7;
    return 16u * (unsigned)(64 * (L >> 3) + 9 * a);
}


//
// Chunks: with K > 1 the lines are solved in K independent chunks of rows
// [floor(k n / K), floor((k+1) n / K)), chunk k by the workgroups of grid row k, with
// tables whose rows couple nothing across a chunk's end (the chunk factors of the
// partitioned solve).  Rows past the end of a chunk then read the next chunk's factor
// rows; they compute values that are never stored and, since the chunk's last rows have
// no coupling beyond it, never reach a stored row.
template <int P, bool CONTIG, int HALVES>
__global__ __launch_bounds__(64 * kSegMaxWaves) void ads_seg_kernel(const double* __restrict__ F,
                                                                     const double* __restrict__ B, int n, int K,
                                                                     long long lines, long long inner,
                                                                     const double* b, double* x)
{
    static_assert(HALVES == 1 || HALVES == 2, "one or two halves per wave");
    constexpr int FR = P + 1, S = kSeg, LPW = 64 / HALVES;   // lines per workgroup
    __shared__ double hand[P][64];
    extern __shared__ __attribute__((aligned(16))) char ads_stage[];   // CONTIG: nw * kStageBytes
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    const int h = HALVES == 2 ? lane >> 5 : 0;                                // half of the line
    const int slot = lane % LPW;                                              // line of the group
    const long long t0 = (long long)blockIdx.x * LPW;
    const long long t = t0 + slot;
    const bool live = t < lines;
    const long long tl = live ? t : lines - 1;
    const long long o = tl / inner, i = tl - o * inner;
    const long long o0 = t0 / inner, i0 = t0 - o0 * inner;
    // rows [cb, cb + len) of the lines (the whole lines when K = 1; the host keeps
    // (K + 1) n below 2^32)
    const int cb = (int)(blockIdx.y * (unsigned)n / (unsigned)K);
    const int len = (int)((blockIdx.y + 1u) * (unsigned)n / (unsigned)K) - cb;
    F += (size_t)cb * FR;
    B += (size_t)cb * FR;
    // rows of this lane: [r0, r0 + S); the wave's first half starts at rw
    const int rw = w * S, r0 = (h * nw + w) * S;
    // wave base: row rw of line t0; lane offset in bytes; row stride in bytes
    const long long wbase = (o0 * (long long)n + cb + rw) * inner + i0;
    const long long total = lines * (long long)n;
    const unsigned voff =
        (unsigned)(((o - o0) * (long long)n * inner + (i - i0) + (long long)(r0 - rw) * inner) * 8);
    const unsigned rstride = (unsigned)(inner * 8);
    const long long left = (total - wbase) * 8;
    const int nrec = (int)(left > 0xffffffffll ? 0xffffffffll : left);
    const auto rb = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(b + wbase), (short)0, nrec, 0x00020000);
    const auto rx = __builtin_amdgcn_make_buffer_rsrc(x + wbase, (short)0, nrec, 0x00020000);
    const int last = len - 1 - r0;   // rows s > last of this lane lie past the end of its line

    // factor rows of one half's segment of this wave, lane s holding row (half nw + w) S + s
    // (zero rows past n)
    double fl[FR], bl[FR];
    auto load_factors = [&](int half) {
        const size_t rl = (size_t)((half * nw + w) * S + min(lane, S - 1)) * FR;
#pragma unroll
        for (int k = 0; k < FR; ++k) {
            fl[k] = F[rl + k];
            bl[k] = B[rl + k];
        }
    };
    load_factors(0);
    // CONTIG staging: this wave's stage; segment L (the rows of lane L) starts seg_off(L)
    // bytes after the wave base, and lane 8a + b of a transfer moves pair b ^ a
    char* const stg = ads_stage + (size_t)w * kStageBytes;
    const int ga = lane >> 3, gj = (lane & 7) ^ (lane >> 3);
    const unsigned own = stage_pos(lane);
    auto seg_off = [&](int L) -> unsigned {
        return (unsigned)(((L % LPW) * n + (L / LPW) * nw * S) * 8);
    };
    double v[S];
    if constexpr (CONTIG) {
        // x-lines (inner = 1).  Pairs that start past the end of a line, and lines past the
        // last, are not read (their stage slots keep stale values, cleared below or never
        // stored); the second row of a pair that ends a line is read and cleared.
#pragma unroll
        for (int c = 0; c < S / kStageRows; ++c) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int L = 8 * q + ga;
                const bool rd = t0 + L % LPW < lines &&
                                c * kStageRows + 2 * gj <= len - 1 - ((L / LPW) * nw + w) * S;
                if (rd)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rb, (__attribute__((address_space(3))) void*)(stg + 1024 * q), 16,
                        (int)(seg_off(L) + 16u * gj), c * kStageRows * 8, 0, 0);
            }
            wait_vm_all();
            wave_lds_order();
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const dv2s d = *reinterpret_cast<const dv2s*>(stg + (own ^ (16u * j)));
                v[c * kStageRows + 2 * j] = d.x;
                v[c * kStageRows + 2 * j + 1] = d.y;
            }
            wait_lds_all();
            wave_lds_order();
        }
    } else if constexpr (HALVES == 1) {
        // the wave's rows end together: the row offset steps in a scalar register, clamped
        // to the last row of the lines
        unsigned so = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            v[s] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rb, (int)voff, (int)so, 0));
            so = opaque_val(s + 1 <= last ? so + rstride : so);
        }
    } else {
        // the halves end at different rows: a row past a lane's line is not read
        unsigned so = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            v[s] = s <= last ? __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rb, (int)voff,
                                                                                                   (int)so, 0))
                             : 0.0;
            so = opaque_val(so + rstride);
        }
    }
    // rows past the end of the lines start from 0 (their factor rows are 0 too), whatever
    // was read for them
#pragma unroll
    for (int s = 0; s < S; ++s) v[s] = s <= last ? v[s] : 0.0;

    // forward: y_r = b_r d_r - sum_k F(r, k) y_{r-P+k}; phase k runs wave k % nw on half
    // k / nw, handing the last P values of each line to the next phase through LDS
    for (int k = 0; k < HALVES * nw; ++k) {
        const int kw = k % nw, kh = k / nw;
        if (w == kw) {
            if (HALVES == 2 && kh == 1) load_factors(1);
            if (h == kh) {
                double yw[P];
#pragma unroll
                for (int j = 0; j < P; ++j) yw[j] = k > 0 ? hand[j][slot] : 0.0;
#pragma unroll
                for (int s = 0; s < S; ++s) {   // rows past the end meet zero factor rows: y = 0
                    double fc[FR];
#pragma unroll
                    for (int j = 0; j <= P; ++j) fc[j] = lane_value(fl[j], s);
                    double y = v[s] * fc[P];
#pragma unroll
                    for (int j = 0; j < P; ++j) y = fma(-fc[j], yw[j], y);
                    v[s] = y;
#pragma unroll
                    for (int j = 0; j + 1 < P; ++j) yw[j] = yw[j + 1];
                    yw[P - 1] = y;
                }
#pragma unroll
                for (int j = 0; j < P; ++j) hand[j][slot] = yw[j];
            }
        }
        __syncthreads();
    }
    // backward: x_r = y_r d_r - sum_{j=1..P} B(r, j-1) x_{r+j}, phases in reverse order
    for (int k = HALVES * nw - 1; k >= 0; --k) {
        const int kw = k % nw, kh = k / nw;
        if (w == kw) {
            if (HALVES == 2 && kh == 0) load_factors(0);
            if (h == kh) {
                double xw[P];   // xw[j-1] = x_{r+j}
#pragma unroll
                for (int j = 0; j < P; ++j) xw[j] = k < HALVES * nw - 1 ? hand[j][slot] : 0.0;
#pragma unroll
                for (int s = S - 1; s >= 0; --s) {   // padded rows meet zero rows: x = 0
                    double bc[FR];
#pragma unroll
                    for (int j = 0; j <= P; ++j) bc[j] = lane_value(bl[j], s);
                    double xv = v[s] * bc[P];
#pragma unroll
                    for (int j = P; j >= 1; --j) xv = fma(-bc[j - 1], xw[j - 1], xv);
                    v[s] = xv;
#pragma unroll
                    for (int j = P - 1; j >= 1; --j) xw[j] = xw[j - 1];
                    xw[0] = xv;
                }
#pragma unroll
                for (int j = 0; j < P; ++j) hand[j][slot] = xw[j];
                if constexpr (!CONTIG) {
                    if (live) {
                        // offsets recomputed here rather than kept from the loads
                        unsigned so = 0;
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            if (s <= last)
                                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(iv2s, v[s]), rx,
                                                                      (int)voff, (int)so, 0);
                            so = opaque_val(so + rstride);
                        }
                    }
                }
            }
            if constexpr (CONTIG) {
                // once both halves of the wave are final (the first half's phase comes
                // last), every lane stages its rows and the wave stores them segment-wise.
                // The transfer lanes' segment, pair and stage position come from the lane
                // index anew rather than being kept live from the loads.
                if (kh == 0) {
                    unsigned ln = threadIdx.x;
                    asm volatile("" : "+v"(ln));
                    ln &= 63u;
                    const unsigned sa = ln >> 3, sj = (ln & 7u) ^ sa, sown = stage_pos((int)ln);
#pragma unroll
                    for (int c = 0; c < S / kStageRows; ++c) {
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            dv2s d;
                            d.x = v[c * kStageRows + 2 * j];
                            d.y = v[c * kStageRows + 2 * j + 1];
                            *reinterpret_cast<dv2s*>(stg + (sown ^ (16u * j))) = d;
                        }
                        wave_lds_order();
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const dv2s d = *reinterpret_cast<const dv2s*>(stg + 16 * (64 * q + ln));
                            const unsigned L = 8u * q + sa;
                            const int s = c * kStageRows + 2 * (int)sj;
                            const int lastL = len - 1 - ((int)(L / LPW) * nw + w) * S;
                            const bool liveL = t0 + (long long)(L % LPW) < lines;
                            const int off = (int)(seg_off((int)L) + 16u * sj);
                            if (liveL && s + 1 <= lastL)
                                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(iv4s, d), rx, off,
                                                                       c * kStageRows * 8, 0);
                            if (liveL && s == lastL)
                                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(iv2s, d.x), rx, off,
                                                                      c * kStageRows * 8, 0);
                        }
                        wait_lds_all();
                        wave_lds_order();
                    }
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace iga
