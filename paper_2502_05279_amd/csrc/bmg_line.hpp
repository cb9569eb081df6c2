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
// be D).  A half-sweep has only n/2 lines and each line is a sequential
// recurrence, so the loads, not the arithmetic, set the pace: one wave serves
// LINE_G lines, all 64 lanes stream chunks of LINE_R rows of them into LDS (the next
// chunk requested while the current one computes), LINE_G lanes run the
// recurrences from LDS, and all lanes write the results back.
constexpr int LINE_G = 4;     // lines per wave
constexpr int LINE_R = 128;   // rows per chunk

static __global__ __launch_bounds__(64) void k_line_solve(int n, int ld, int par, double *__restrict__ D,
                                                          const double *__restrict__ lf,
                                                          const double *__restrict__ rf,
                                                          const double *__restrict__ C, double *X,
                                                          const int *stop)
{
    if (stopped(stop)) return;
    __shared__ double buf[2][3][LINE_R][LINE_G];
    constexpr int PL = LINE_R / (64 / LINE_G);               // rows each lane moves per chunk
    const int lane = threadIdx.x;
    const int t = lane % LINE_G, q = lane / LINE_G;          // moving: line t, rows q, q + 8, ...
    const int nlines = par ? (n + 1) / 2 : (n - 1) / 2;
    const int line0 = blockIdx.x * LINE_G;
    const bool lok = line0 + t < nlines;
    const size_t col = (size_t)((par ? 1 : 2) + 2 * (line0 + t));
    const size_t sld = ld;
    const bool comp = lane < LINE_G && line0 + lane < nlines;   // computing: line `lane`
    const int nch = (n + LINE_R - 1) / LINE_R;

    // forward over rows 1..n: y_1 = d_1, y_k = d_k - l_k y_{k-1}
    double rd[PL], rl[PL];
    auto fload = [&](int ch) {
#pragma unroll
        for (int s = 0; s < PL; ++s) {
            const int k = 1 + ch * LINE_R + q + (64 / LINE_G) * s;
            const bool ok = lok && k <= n;
            const size_t p = ok ? (size_t)k * sld + col : 0;
            rd[s] = ok ? D[p] : 0.0;
            rl[s] = ok ? lf[p] : 0.0;
        }
    };
    auto fput = [&](int b) {
#pragma unroll
        for (int s = 0; s < PL; ++s) {
            buf[b][0][q + (64 / LINE_G) * s][t] = rd[s];
            buf[b][1][q + (64 / LINE_G) * s][t] = rl[s];
        }
    };
    fload(0);
    fput(0);
    __syncthreads();
    double y = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
        const int b = ch & 1;
        if (ch + 1 < nch) fload(ch + 1);
        if (comp) {
            // sub-blocks of 16 rows: their LDS reads are issued together, so
            // only the recurrence's own arithmetic is sequential
            for (int r0 = 0; r0 < LINE_R && 1 + ch * LINE_R + r0 <= n; r0 += 16) {
                double dv[16], lv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    dv[u] = buf[b][0][r0 + u][lane];
                    lv[u] = buf[b][1][r0 + u][lane];
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int k = 1 + ch * LINE_R + r0 + u;
                    if (k <= n) {
                        y = k == 1 ? dv[u] : dv[u] - lv[u] * y;
                        buf[b][0][r0 + u][lane] = y;
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PL; ++s) {
            const int k = 1 + ch * LINE_R + q + (64 / LINE_G) * s;
            if (lok && k <= n) D[(size_t)k * sld + col] = buf[b][0][q + (64 / LINE_G) * s][t];
        }
        if (ch + 1 < nch) fput(b ^ 1);
        __syncthreads();
    }

    // back over rows n..1: x_n = y_n r_n, x_k = (y_k - c_k x_{k+1}) r_k
    double ry[PL], rr[PL], rc[PL];
    auto bload = [&](int ch) {   // chunk ch from the top: rows n - ch LINE_R - (0 .. LINE_R-1)
#pragma unroll
        for (int s = 0; s < PL; ++s) {
            const int k = n - ch * LINE_R - q - (64 / LINE_G) * s;
            const bool ok = lok && k >= 1;
            const size_t p = ok ? (size_t)k * sld + col : 0;
            ry[s] = ok ? D[p] : 0.0;
            rr[s] = ok ? rf[p] : 0.0;
            rc[s] = ok ? C[p + sld] : 0.0;
        }
    };
    auto bput = [&](int b) {
#pragma unroll
        for (int s = 0; s < PL; ++s) {
            buf[b][0][q + (64 / LINE_G) * s][t] = ry[s];
            buf[b][1][q + (64 / LINE_G) * s][t] = rr[s];
            buf[b][2][q + (64 / LINE_G) * s][t] = rc[s];
        }
    };
    bload(0);
    bput(0);
    __syncthreads();
    double x = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
        const int b = ch & 1;
        if (ch + 1 < nch) bload(ch + 1);
        if (comp) {
            for (int r0 = 0; r0 < LINE_R && n - ch * LINE_R - r0 >= 1; r0 += 16) {
                double yv[16], rv[16], cv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    yv[u] = buf[b][0][r0 + u][lane];
                    rv[u] = buf[b][1][r0 + u][lane];
                    cv[u] = buf[b][2][r0 + u][lane];
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int k = n - ch * LINE_R - r0 - u;
                    if (k >= 1) {
                        x = k == n ? yv[u] * rv[u] : (yv[u] - cv[u] * x) * rv[u];
                        buf[b][0][r0 + u][lane] = x;
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PL; ++s) {
            const int k = n - ch * LINE_R - q - (64 / LINE_G) * s;
            if (lok && k >= 1) X[(size_t)k * sld + col] = buf[b][0][q + (64 / LINE_G) * s][t];
        }
        if (ch + 1 < nch) bput(b ^ 1);
        __syncthreads();
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
