// Line relaxation: alternating zebra line Gauss-Seidel (the "Line" relaxation
// of Fig. vcycle_flowchart).  One relaxation solves the x-lines (rows) of odd
// index, then of even index, then the y-lines (columns) of odd and of even
// index; each line's equations are solved exactly with the other unknowns at
// their current values.  A line is tridiagonal:
//   x-line j: a_i = A_W(i,j), b_i = A_O(i,j), c_i = A_E(i,j);
//   y-line i: a_j = A_S(i,j), b_j = A_O(i,j), c_j = A_N(i,j);
// its right-hand side is b minus the couplings to the neighbouring lines, the
// lower (x: SW, S, SE) or left (y: SW, W, NW) one first, then the upper
// (NW, N, NE) or right (SE, E, NE) one.  With this order an x-line is the
// y-line of the transposed grid, so one column kernel solves both: x-lines
// run on transposed copies (element (i, j) at i*ld + j) of their right-hand
// side, factor and coupling.
//
// Each line matrix is factored at set-up, T = L U: m_1 = b_1,
// l_k = a_k / m_{k-1}, m_k = b_k - l_k a_k (the matrix is symmetric, so
// c_{k-1} = a_k), keeping l_k and the reciprocal pivot r_k = 1 / m_k.  A solve
// is y_1 = d_1, y_k = d_k - l_k y_{k-1}; x_n = y_n r_n,
// x_k = (y_k - c_k x_{k+1}) r_k.
#pragma once

#include "bmg_kernels.hpp"

namespace bmg {

constexpr int LT = 32;  // tile side of the transposes

// Factor of the columns of a level in the frame of the arrays given: O the
// diagonal, A the coupling of (c, k) to (c, k-1) (S, or the transposed W).
static __global__ void k_line_factor(int n, int ld, const double *__restrict__ O, const double *__restrict__ A,
                                     double *__restrict__ lf, double *__restrict__ rf, int *__restrict__ flags)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (c > n) return;
    double m_prev = 0.0;
    int bad = 0;
    for (int k = 1; k <= n; ++k) {
        const size_t p = (size_t)k * ld + c;
        double m;
        if (k == 1) {
            lf[p] = 0.0;
            m = O[p];
        } else {
            const double a = A[p];
            const double l = a / m_prev;
            lf[p] = l;
            m = O[p] - l * a;
        }
        if (!(m > 0.0) || !isfinite(m)) bad = 1;
        rf[p] = 1.0 / m;
        m_prev = m;
    }
    if (bad) atomicOr(flags, F_BREAK_LINE);
}

// dst(i, j) = src(j, i) over the whole (n+2) x (n+2) array, 32 x 32 tiles
// through LDS (both sides coalesced).
static __global__ void k_transpose(int n, int ld, const double *__restrict__ src, double *__restrict__ dst)
{
    __shared__ double t[LT][LT + 1];
    const int bi = blockIdx.x * LT, bj = blockIdx.y * LT;
    for (int r = threadIdx.y; r < LT; r += blockDim.y) {
        const int i = bi + threadIdx.x, j = bj + r;
        if (i <= n + 1 && j <= n + 1) t[r][threadIdx.x] = src[(size_t)j * ld + i];
    }
    __syncthreads();
    for (int r = threadIdx.y; r < LT; r += blockDim.y) {
        const int j = bj + threadIdx.x, i = bi + r;
        if (i <= n + 1 && j <= n + 1) dst[(size_t)i * ld + j] = t[threadIdx.x][r];
    }
}

// Right-hand sides of the y-lines (columns) of parity `par` into D.
template <bool NINE>
static __global__ void k_line_rhs_y(Lev<double> L, int par, double *__restrict__ D, const int *stop)
{
    if (stopped(stop)) return;
    const int i = 2 * (blockIdx.x * blockDim.x + threadIdx.x) + (par ? 1 : 2);
    const int j = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (i > L.n || j > L.n) return;
    const size_t ld = L.ld, p = (size_t)j * ld + i;
    const double *u = L.u;
    double d = L.b[p];
    if (NINE) d -= L.SW[p] * u[p - ld - 1];
    d -= L.W[p] * u[p - 1];
    if (NINE) d -= L.NW[p] * u[p + ld - 1];
    if (NINE) d -= L.NW[p + 1 - ld] * u[p - ld + 1];   // A_SE
    d -= L.W[p + 1] * u[p + 1];                        // A_E
    if (NINE) d -= L.SW[p + ld + 1] * u[p + ld + 1];   // A_NE
    D[p] = d;
}

// Right-hand sides of the x-lines (rows) of parity `par`, written transposed
// into DT (element (i, j) at i*ld + j) through an LDS tile.
template <bool NINE>
static __global__ void k_line_rhs_x(Lev<double> L, int par, double *__restrict__ DT, const int *stop)
{
    if (stopped(stop)) return;
    __shared__ double t[LT][LT + 1];
    const int bi = blockIdx.x * LT, bj = blockIdx.y * LT;
    const size_t ld = L.ld;
    const double *u = L.u;
    for (int r = threadIdx.y; r < LT; r += blockDim.y) {
        const int i = bi + threadIdx.x, j = bj + r;
        if (i >= 1 && i <= L.n && j >= 1 && j <= L.n && (j & 1) == par) {
            const size_t p = (size_t)j * ld + i;
            double d = L.b[p];
            if (NINE) d -= L.SW[p] * u[p - ld - 1];
            d -= L.S[p] * u[p - ld];
            if (NINE) d -= L.NW[p + 1 - ld] * u[p - ld + 1];   // A_SE
            if (NINE) d -= L.NW[p] * u[p + ld - 1];
            d -= L.S[p + ld] * u[p + ld];                      // A_N
            if (NINE) d -= L.SW[p + ld + 1] * u[p + ld + 1];   // A_NE
            t[r][threadIdx.x] = d;
        }
    }
    __syncthreads();
    for (int r = threadIdx.y; r < LT; r += blockDim.y) {
        const int j = bj + threadIdx.x, i = bi + r;
        if (i >= 1 && i <= L.n && j >= 1 && j <= L.n && (j & 1) == par) DT[(size_t)i * ld + j] = t[threadIdx.x][r];
    }
}

// Solve of the columns of parity `par` in the frame of the arrays given: the
// right-hand side in D (overwritten by y), the factor lf, rf, the coupling
// C(c, k) = c_k (A_N, or the transposed A_E); the solution into X (which may
// be D).  One lane per column; the rows stream in order, coalesced, in blocks
// of LINE_BLK whose loads are requested while the previous block computes (a
// half-sweep has only n/2 lines, so each lane must keep many loads in flight).
constexpr int LINE_BLK = 16;

static __global__ __launch_bounds__(64) void k_line_solve(int n, int ld, int par, double *__restrict__ D,
                                                          const double *__restrict__ lf,
                                                          const double *__restrict__ rf,
                                                          const double *__restrict__ C, double *X,
                                                          const int *stop)
{
    if (stopped(stop)) return;
    const int c = 2 * (blockIdx.x * blockDim.x + threadIdx.x) + (par ? 1 : 2);
    if (c > n) return;
    const size_t sld = ld;
    // forward: y_1 = d_1, y_k = d_k - l_k y_{k-1}, over rows 1..n
    double dv[LINE_BLK], lv[LINE_BLK], dn[LINE_BLK], ln[LINE_BLK];
    auto fload = [&](int k0, double *d, double *l) {
#pragma unroll
        for (int t = 0; t < LINE_BLK; ++t) {
            const int k = k0 + t;
            const size_t p = (size_t)(k <= n ? k : n) * sld + c;
            d[t] = D[p];
            l[t] = lf[p];
        }
    };
    fload(1, dv, lv);
    double y = 0.0;
    for (int k0 = 1; k0 <= n; k0 += LINE_BLK) {
        if (k0 + LINE_BLK <= n) fload(k0 + LINE_BLK, dn, ln);
#pragma unroll
        for (int t = 0; t < LINE_BLK; ++t) {
            const int k = k0 + t;
            if (k <= n) {
                y = k == 1 ? dv[t] : dv[t] - lv[t] * y;
                D[(size_t)k * sld + c] = y;
            }
        }
#pragma unroll
        for (int t = 0; t < LINE_BLK; ++t) { dv[t] = dn[t]; lv[t] = ln[t]; }
    }
    // back: x_n = y_n r_n, x_k = (y_k - c_k x_{k+1}) r_k, over rows n..1
    double yv[LINE_BLK], rv[LINE_BLK], cv[LINE_BLK], yn[LINE_BLK], rn[LINE_BLK], cn[LINE_BLK];
    auto bload = [&](int k0, double *yy, double *r, double *cc) {   // rows k0, k0-1, ...
#pragma unroll
        for (int t = 0; t < LINE_BLK; ++t) {
            const int k = k0 - t;
            const size_t p = (size_t)(k >= 1 ? k : 1) * sld + c;
            yy[t] = D[p];
            r[t] = rf[p];
            cc[t] = C[p + sld];
        }
    };
    bload(n, yv, rv, cv);
    double x = 0.0;
    for (int k0 = n; k0 >= 1; k0 -= LINE_BLK) {
        if (k0 - LINE_BLK >= 1) bload(k0 - LINE_BLK, yn, rn, cn);
#pragma unroll
        for (int t = 0; t < LINE_BLK; ++t) {
            const int k = k0 - t;
            if (k >= 1) {
                x = k == n ? yv[t] * rv[t] : (yv[t] - cv[t] * x) * rv[t];
                X[(size_t)k * sld + c] = x;
            }
        }
#pragma unroll
        for (int t = 0; t < LINE_BLK; ++t) { yv[t] = yn[t]; rv[t] = rn[t]; cv[t] = cn[t]; }
    }
}

// u(i, j) = XT(j, i) ... the transposed x-line solutions back into the rows of
// parity `par`.
static __global__ void k_line_put_x(int n, int ld, int par, const double *__restrict__ XT, double *__restrict__ u,
                                    const int *stop)
{
    if (stopped(stop)) return;
    __shared__ double t[LT][LT + 1];
    const int bi = blockIdx.x * LT, bj = blockIdx.y * LT;
    // read XT rows i (transposed frame), columns j, coalesced along j
    for (int r = threadIdx.y; r < LT; r += blockDim.y) {
        const int i = bi + r, j = bj + threadIdx.x;
        if (i >= 1 && i <= n && j >= 1 && j <= n && (j & 1) == par) t[r][threadIdx.x] = XT[(size_t)i * ld + j];
    }
    __syncthreads();
    for (int r = threadIdx.y; r < LT; r += blockDim.y) {
        const int j = bj + r, i = bi + threadIdx.x;
        if (i >= 1 && i <= n && j >= 1 && j <= n && (j & 1) == par) u[(size_t)j * ld + i] = t[threadIdx.x][r];
    }
}

}  // namespace bmg
