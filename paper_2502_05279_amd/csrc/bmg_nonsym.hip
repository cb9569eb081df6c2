// Nonsymmetric black-box multigrid on the GPU (gfx950): the BoxMG variant for
// operators with A != A^T (convection-diffusion).  The interpolation P is
// induced by A as in the symmetric solver; the restriction is the transpose of
// the interpolation induced by A^T; the coarse operators are the
// Petrov-Galerkin products R A P in all nine directions; the coarsest level is
// factored as a band L D U and solved by the same one-wave band kernel as the
// symmetric solver.  Every level keeps all nine entries of each row.  The
// cycle runs the unfused steps (one launch per colour, residual, restriction,
// interpolation), each point's expressions in the order of the oracle, so the
// iterates are the oracle's to the bit.
#include "bmg_internal.hpp"

#include <math.h>
#include <string.h>

#include <algorithm>

using namespace bmgi;

namespace {

constexpr int NSD = 9;   // stencil entries SW, S, SE, W, O, E, NW, N, NE
enum : int { E_SW = 0, E_S, E_SE, E_W, E_O, E_E, E_NW, E_N, E_NE };

// A level: nine padded planes of (n+2) rows of pitch ld, A[e][p] the coupling of
// row p to p + d(e), zero on the Dirichlet ring.
struct LevN {
    int n, ld;
    double *A[NSD];
    double *u, *b, *r;
};

__device__ __forceinline__ ptrdiff_t ns_off(int e, int ld) { return (e % 3 - 1) + (ptrdiff_t)(e / 3 - 1) * ld; }

// Row p of A, or of A^T (A^T(p, p + d) = A(p + d, p), entry 8 - e of row p + d).
__device__ __forceinline__ void ns_row(const LevN &L, size_t p, bool transpose, double a[NSD])
{
#pragma unroll
    for (int e = 0; e < NSD; ++e)
        a[e] = (!transpose || e == E_O) ? L.A[e][p] : L.A[NSD - 1 - e][(size_t)((ptrdiff_t)p + ns_off(e, L.ld))];
}

// [n][n][K] stencil (K = 5: S, W, O, E, N; K = 9: SW..NE) into level 0, with
// the validation bits of the symmetric import (no symmetry check).
__global__ void k_ns_import(const double *__restrict__ st, int K, LevN L, int *__restrict__ flags)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const int n = L.n;
    const size_t p = (size_t)j * L.ld + i;
    const double *q = st + ((size_t)(j - 1) * n + (i - 1)) * K;
    int bad = 0;
    for (int t = 0; t < K; ++t) {
        const int e = K == 5 ? (t == 0 ? E_S : t == 1 ? E_W : t == 2 ? E_O : t == 3 ? E_E : E_N) : t;
        const double v = q[t];
        if (!isfinite(v)) bad |= F_NONFINITE;
        if (e == E_O && !(v > 0.0)) bad |= F_DIAG;
        const int qi = i + e % 3 - 1, qj = j + e / 3 - 1;
        if (e != E_O && (qi < 1 || qi > n || qj < 1 || qj > n) && v != 0.0) bad |= F_BOUNDARY;
        L.A[e][p] = v;
    }
    if (bad) atomicOr(flags, bad);
}

// Operator-induced edge weights of A (transpose = false: P) or of A^T (R's
// weights), the formulas of the symmetric solver on the lumped rows.
__global__ void k_ns_weights_edges(LevN F, Wts<double> C, int nc, bool transpose, int *__restrict__ flags)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int J = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (I > nc + 1 || J > nc + 1) return;
    const size_t c = (size_t)J * C.ld + I;
    const size_t ld = F.ld;
    int bad = 0;
    double a[NSD];
    if (J <= nc) {
        ns_row(F, (size_t)(2 * J) * ld + (2 * I - 1), transpose, a);
        lump_row(a);
        const double D = (a[E_O] + a[E_N]) + a[E_S];
        if (!(D > 0.0)) bad = F_BREAK_INTERP;
        C.p[LL * C.ps + c] = -((a[E_W] + a[E_NW]) + a[E_SW]) / D;
        C.p[LR * C.ps + c] = -((a[E_E] + a[E_NE]) + a[E_SE]) / D;
    }
    if (I <= nc) {
        ns_row(F, (size_t)(2 * J - 1) * ld + (2 * I), transpose, a);
        lump_row(a);
        const double D = (a[E_O] + a[E_W]) + a[E_E];
        if (!(D > 0.0)) bad = F_BREAK_INTERP;
        C.p[LB * C.ps + c] = -((a[E_S] + a[E_SW]) + a[E_SE]) / D;
        C.p[LA * C.ps + c] = -((a[E_N] + a[E_NW]) + a[E_NE]) / D;
    }
    if (bad) atomicOr(flags, bad);
}

__global__ void k_ns_weights_corners(LevN F, Wts<double> C, int nc, bool transpose, int *__restrict__ flags)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int J = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (I > nc + 1 || J > nc + 1) return;
    const size_t c = (size_t)J * C.ld + I;
    const size_t cs = c - C.ld, cw = c - 1;
    double a[NSD];
    ns_row(F, (size_t)(2 * J - 1) * F.ld + (2 * I - 1), transpose, a);
    lump_row(a);
    if (!(a[E_O] > 0.0)) atomicOr(flags, F_BREAK_INTERP);
    const double lr = C.at(LR, c), ll = C.at(LL, c), la = C.at(LA, c), lb = C.at(LB, c);
    const double lr_s = C.at(LR, cs), ll_s = C.at(LL, cs);
    const double la_w = C.at(LA, cw), lb_w = C.at(LB, cw);
    C.p[LNE * C.ps + c] = -((a[E_NE] + a[E_N] * lr) + a[E_E] * la) / a[E_O];
    C.p[LNW * C.ps + c] = -((a[E_NW] + a[E_N] * ll) + a[E_W] * la_w) / a[E_O];
    C.p[LSE * C.ps + c] = -((a[E_SE] + a[E_S] * lr_s) + a[E_E] * lb) / a[E_O];
    C.p[LSW * C.ps + c] = -((a[E_SW] + a[E_S] * ll_s) + a[E_W] * lb_w) / a[E_O];
}

// A_c(I,J; d) = sum_p R(p; IJ) sum_q A(p, q) P(q; IJ + d) for the nine d, p over
// the fine 3x3 patch (rows south to north), q over p's neighbours SW..NE in the
// support of basis IJ + d; couplings to ring coarse points are zero: their
// sums are formed with the weights of the nearest interior point (so every
// load is in range and none waits behind a branch) and then replaced by zero.
__global__ __launch_bounds__(256) void k_ns_rap(LevN F, Wts<double> P, Wts<double> R, LevN Cl)
{
    const int I = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int J = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    const int nc = Cl.n;
    if (I > nc || J > nc) return;
    const size_t c = (size_t)J * Cl.ld + I;
#pragma unroll
    for (int d = 0; d < NSD; ++d) {
        const int ki = I + d % 3 - 1, kj = J + d / 3 - 1;
        const bool live = ki >= 1 && ki <= nc && kj >= 1 && kj <= nc;
        const int KI = ki < 1 ? 1 : ki > nc ? nc : ki, KJ = kj < 1 ? 1 : kj > nc ? nc : kj;
        double acc = 0.0;
#pragma unroll
        for (int jj = -1; jj <= 1; ++jj) {
#pragma unroll
            for (int ii = -1; ii <= 1; ++ii) {
                const int pi = 2 * I + ii, pj = 2 * J + jj;
                const double wp = basis_weight(R, I, J, ii, jj);
                double a[NSD];
                ns_row(F, (size_t)pj * F.ld + pi, false, a);
                double t = 0.0;
#pragma unroll
                for (int e = 0; e < NSD; ++e) {
                    // q - 2(IJ + d), the same for the clamped point's support
                    const int dx = ii + e % 3 - 1 - 2 * (d % 3 - 1), dy = jj + e / 3 - 1 - 2 * (d / 3 - 1);
                    if (dx < -1 || dx > 1 || dy < -1 || dy > 1) continue;
                    t = t + a[e] * basis_weight(P, KI, KJ, dx, dy);
                }
                acc = acc + wp * t;
            }
        }
        Cl.A[d][c] = live ? acc : 0.0;
    }
}

// s = b - sum of the eight couplings in the order SW, S, SE, W, E, NW, N, NE.
__device__ __forceinline__ double ns_offdiag(const LevN &L, const double *__restrict__ u, size_t p)
{
    double s = L.b[p];
#pragma unroll
    for (int e = 0; e < NSD; ++e) {
        if (e == E_O) continue;
        s -= L.A[e][p] * u[(size_t)((ptrdiff_t)p + ns_off(e, L.ld))];
    }
    return s;
}

// One sweep's two colours of the rows of one parity (rp = 0: the even rows,
// colours 0 and 1; rp = 1: the odd rows, colours 2 and 3), one wave per row.
// The wave walks its row from west to east in chunks of 64 column pairs:
// first the chunk's even columns (the first colour), then its odd columns
// (the second), whose west and east neighbours are the row's new even values
// (the neighbouring lane's, or for lane 0 the last one of the previous
// chunk).  An even point reads the odd values of its own and the next chunk,
// which are not yet written; every other value a point reads lies in rows
// j - 1 and j + 1, which this launch does not write.  So each point sees the
// values, in the order, of one launch per colour, and the stencil rows are
// read once for both colours.
constexpr int NS_PAIR_WAVES = 4;

// The operands of one chunk for one lane: the even point's nine stencil
// entries, eight neighbours and right-hand side, the odd point's nine entries,
// its six neighbours in rows j - 1 and j + 1, and right-hand side.  None of
// them is written by an earlier chunk of the row, so the next chunk's are
// requested before the current one computes.
struct NsPair {
    double ae[NSD], ue[NSD], be, ao[NSD], uo[NSD], bo;
};

__device__ __forceinline__ void ns_pair_load(const LevN &L, size_t row, int g, NsPair &c)
{
    const int n = L.n, ie = 2 + 2 * g, io = 1 + 2 * g;
    const size_t pe = row + ie, po = row + io;
    const bool ev = ie <= n, od = io <= n;
#pragma unroll
    for (int e = 0; e < NSD; ++e) {
        const ptrdiff_t d = ns_off(e, L.ld);
        c.ae[e] = ev ? L.A[e][pe] : 0.0;
        c.ue[e] = ev && e != E_O ? L.u[(size_t)((ptrdiff_t)pe + d)] : 0.0;
        c.ao[e] = od ? L.A[e][po] : 0.0;
        c.uo[e] = od && e != E_O && e != E_W && e != E_E ? L.u[(size_t)((ptrdiff_t)po + d)] : 0.0;
    }
    c.be = ev ? L.b[pe] : 0.0;
    c.bo = od ? L.b[po] : 0.0;
}

__global__ __launch_bounds__(64 * NS_PAIR_WAVES) void k_ns_gs_pair(LevN L, int rp)
{
    const int lane = threadIdx.x & 63, n = L.n;
    const int j = (rp ? 1 : 2) + 2 * (int)(blockIdx.x * NS_PAIR_WAVES + (threadIdx.x >> 6));
    if (j > n) return;   // the whole wave
    const size_t row = (size_t)j * L.ld;
    double carry = L.u[row];   // the ring value west of column 1
    NsPair cur, nxt;
    ns_pair_load(L, row, lane, nxt);
    for (int g0 = 0; 2 * g0 + 1 <= n; g0 += 64) {
        cur = nxt;
        if (2 * (g0 + 64) + 1 <= n) ns_pair_load(L, row, g0 + 64 + lane, nxt);
        const int g = g0 + lane, ie = 2 + 2 * g, io = 1 + 2 * g;
        double ev = 0.0;
        if (ie <= n) {
            // ns_offdiag's terms in its order, then the division
            double s = cur.be;
#pragma unroll
            for (int e = 0; e < NSD; ++e) {
                if (e == E_O) continue;
                s -= cur.ae[e] * cur.ue[e];
            }
            ev = s / cur.ae[E_O];
            L.u[row + ie] = ev;
        } else if (ie == n + 1) {
            ev = L.u[row + ie];   // the ring value east of column n
        }
        double west = __shfl_up(ev, 1);
        if (lane == 0) west = carry;
        carry = __shfl(ev, 63);
        if (io <= n) {
            double s = cur.bo;
#pragma unroll
            for (int e = 0; e < NSD; ++e) {
                if (e == E_O) continue;
                const double x = e == E_W ? west : e == E_E ? ev : cur.uo[e];
                s -= cur.ao[e] * x;
            }
            L.u[row + io] = s / cur.ao[E_O];
        }
    }
}

// r = b - A u, the centre term last.
__global__ void k_ns_residual(LevN L)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const size_t p = (size_t)j * L.ld + i;
    double s = ns_offdiag(L, L.u, p);
    s -= L.A[E_O][p] * L.u[p];
    L.r[p] = s;
}

// ------------------------------------------------ coarsest band L D U
// A = L D U with unit triangular L, U (band of w = nc + 1 on each side of the
// diagonal) in right-looking form: once column k is final (D_k = a_kk,
// L_ik = a_ik / D_k, U_kj = a_kj / D_k), every entry of the trailing window
// takes its term, a_ij <- a_ij - L_ik a_kj (k < i, j <= k + w), so each entry
// receives its terms in increasing k, the products of the definition's
// column-by-column form.  By panels of BAND_PANEL columns, as the symmetric
// factor: wave 0 finishes a panel's columns and rows in registers (lane l
// holds, for the panel, rows k0 + l and k0 + 64 + l of its columns and
// columns k0 + l and k0 + 64 + l of its rows; the band below column k and the
// band right of row k are one entry per lane), with the terms they give to
// the panel's own later columns and rows; then every thread applies the
// panel's terms, in column order, to its entries of the w x w trailing window,
// writes the panel's L, U and D, and the rows the next panel adds enter the
// window (their nine band entries of A requested two panels ahead).  Rows
// live in an LDS ring (row i, column j at slot i mod NSB_RR, offset j - i + w).
// Lb[i w + (k - i + w)] = L_ik, Ub[i w + (k - i - 1)] = U_ik, D.
constexpr int NSB_THREADS = 1024;
constexpr int NSB_RW = 2 * BAND_MAX_NC + 3;            // ring row: offsets 0 .. 2w
constexpr int NSB_RR = BAND_MAX_NC + 1 + BAND_PANEL;   // ring rows: a panel's window
constexpr int NSB_LW = BAND_MAX_NC + 2;                // a panel column's L (row's U) at offsets 1 .. w
static_assert(BAND_PANEL * NSB_RW <= 2 * NSB_THREADS && (BAND_MAX_NC + 1) * (BAND_MAX_NC + 1) <= 4 * NSB_THREADS &&
                  (BAND_MAX_NC + BAND_PANEL) * BAND_PANEL <= NSB_THREADS,
              "entering rows in two passes, the trailing window in four, the panel's L in one");

__host__ __device__ inline size_t ns_band_lds()
{
    return ((size_t)NSB_RR * NSB_RW + 2 * BAND_PANEL * NSB_LW + BAND_PANEL + 2 * BAND_PANEL * NSD) * sizeof(double);
}

__global__ __launch_bounds__(NSB_THREADS) void k_band_ldu_factor(LevN L, double *__restrict__ Lb,
                                                                  double *__restrict__ Ub, double *__restrict__ D,
                                                                  int *__restrict__ flags)
{
    constexpr int B = BAND_PANEL;
    extern __shared__ double nsb_sm[];
    double *ring = nsb_sm;
    double(*Lp)[NSB_LW] = reinterpret_cast<double(*)[NSB_LW]>(ring + NSB_RR * NSB_RW);   // L(k + d, k)
    double(*Up)[NSB_LW] = Lp + B;                                                         // a(k, k + d)
    double *Dpan = reinterpret_cast<double *>(Up + B);
    double *stage = Dpan + B;   // [2][B * NSD]
    const int nc = L.n, m = nc * nc, w = nc + 1, t = threadIdx.x;
    const int npanel = (m + B - 1) / B;
    auto at = [&](int i, int j) -> double & { return ring[(i % NSB_RR) * NSB_RW + (j - i + w)]; };
    // A(i, i + off(e)) for the nine entries of row i (zero outside the grid)
    auto entry = [&](int i, int e) -> double {
        const int ii = i % nc + 1, jj = i / nc + 1, qi = ii + e % 3 - 1, qj = jj + e / 3 - 1;
        if (qi < 1 || qi > nc || qj < 1 || qj > nc) return 0.0;
        return L.A[e][(size_t)jj * L.ld + ii];
    };
    auto col_of = [&](int i, int e) { return i + (e % 3 - 1) + (e / 3 - 1) * nc; };
    // rows 0 .. w + B - 1 (the window of panel 0)
    for (int e2 = t; e2 < (w + B) * (2 * w + 1); e2 += blockDim.x) {
        const int i = e2 / (2 * w + 1), off = e2 % (2 * w + 1);
        if (i < m) at(i, i - w + off) = 0.0;
    }
    lds_barrier();
    for (int e2 = t; e2 < (w + B) * NSD; e2 += blockDim.x) {
        const int i = e2 / NSD, e = e2 % NSD;
        if (i < m) at(i, col_of(i, e)) = entry(i, e);
    }
    // the rows panel q adds to the window: q B + w .. q B + w + B - 1; entry u
    // of its staging buffer is row q B + w + u / NSD, direction u % NSD
    auto entering = [&](int q, int u) -> double {
        const int i = q * B + w + u / NSD;
        return i < m ? entry(i, u % NSD) : 0.0;
    };
    const bool loader = t < B * NSD;
    if (loader) stage[B * NSD + t] = entering(1, t);
    double pf = loader ? entering(2, t) : 0.0;        // panel 2's rows, in flight
    // this thread's slots of the rows entering the window (row eb, offset
    // eoff; eu: its staging entry, -1 for a zero of the band)
    int eb[2], eoff[2], eu[2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
        const int e = t + s2 * NSB_THREADS;
        eb[s2] = e < B * (2 * w + 1) ? e / (2 * w + 1) : -1;
        eoff[s2] = e % (2 * w + 1);
        eu[s2] = -1;
#pragma unroll
        for (int d = 0; d < NSD; ++d)
            if (eoff[s2] - w == (d % 3 - 1) + (d / 3 - 1) * nc) eu[s2] = eb[s2] * NSD + d;
    }
    int bad = 0;
    lds_barrier();
    for (int p = 0; p < npanel; ++p) {
        const int k0 = p * B;
        if (t < 64) {
            // wave 0.  L view: rows r0 = k0 + l, r1 = k0 + 64 + l of the panel's
            // columns; U view: columns r0, r1 of the panel's rows.  The rows
            // below column k = k0 + b within the band are the first row of
            // lanes l > b and the second row of lanes l <= b (and so for the
            // columns right of row k); outside the band an entry holds zero
            // and takes zero terms, rows and columns past the matrix act as
            // those of the identity, and entries on the wrong side of the
            // diagonal take terms that are never read
            // the lane index, opaque to the compiler here, so that the
            // per-column addresses and tests below are formed in each panel
            // rather than kept (and spilled) across the loop
            int ln = t;
            asm volatile("" : "+v"(ln));
            const int r0 = k0 + ln, r1 = k0 + 64 + ln;
            double a0[B], a1[B], u0[B], u1[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int k = k0 + b;
                a0[b] = r0 >= m ? (r0 == k ? 1.0 : 0.0) : (r0 >= k && r0 - k <= w) ? at(r0, k) : 0.0;
                a1[b] = (r1 < m && r1 - k <= w) ? at(r1, k) : 0.0;
                u0[b] = (r0 < m && r0 > k && r0 - k <= w) ? at(k, r0) : 0.0;
                u1[b] = (r1 < m && r1 - k <= w) ? at(k, r1) : 0.0;
            }
            double dg = 0.0;   // D of the lane's own panel column
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const double Dk = readlane_d(a0[b], b);
                dg = ln == b ? a0[b] : dg;
                const bool first = ln > b;
                const double l = (first ? a0[b] : a1[b]) / Dk;
                const double uv = first ? u0[b] : u1[b];
                const int d = first ? ln - b : 64 + ln - b;   // the lane's row and column of k are k + d
                if (d <= w) {
                    Lp[b][d] = l;
                    Up[b][d] = uv;
                }
                const double l1 = first ? 0.0 : l;
                // the terms of column and row k in the panel's later columns and rows
#pragma unroll
                for (int jb = b + 1; jb < B; ++jb) {
                    const double vj = readlane_d(u0[b], jb);   // a(k, k0 + jb)
                    const double lj = readlane_d(l, jb);       // L(k0 + jb, k)
                    a0[jb] = a0[jb] - l * vj;
                    a1[jb] = a1[jb] - l1 * vj;
                    u0[jb] = u0[jb] - lj * u0[b];
                    u1[jb] = u1[jb] - lj * u1[b];
                }
            }
            if (t < B) Dpan[t] = dg;
        }
        lds_barrier();
        // the panel's L, U and D to memory
        if (t < (w + B - 1) * B) {
            const int r = k0 + 1 + t / B, b = t % B, d = r - k0 - b;
            if (d >= 1 && d <= w && r < m) Lb[(size_t)r * w + (w - d)] = Lp[b][d];
        }
        if (t < B * w) {
            const int b = t / w, d = 1 + t % w, k = k0 + b;
            if (k + d < m) Ub[(size_t)k * w + (d - 1)] = Up[b][d] / Dpan[b];
        }
        if (t >= NSB_THREADS - B) {
            const int b = t - (NSB_THREADS - B);
            if (k0 + b < m) {
                const double Dk = Dpan[b];
                D[k0 + b] = Dk;
                if (!(Dk > 0.0)) bad = 1;
            }
        }
        // the panel's terms in the trailing window (rows and columns
        // k0 + B .. k0 + B - 1 + w), in column order
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            const int e = t + s2 * NSB_THREADS;
            const int i = k0 + B + e / w, j = k0 + B + e % w;
            if (e < w * w && i < m && j < m) {
                double a = at(i, j);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int k = k0 + b;
                    if (i - k <= w && j - k <= w && k < m) a = a - Lp[b][i - k] * Up[b][j - k];
                }
                at(i, j) = a;
            }
        }
        // the rows of panel p + 1 enter (their slots are those of panel p's
        // rows); the staging buffer of panel p + 2 is filled from the
        // registers and panel p + 3's entries are requested
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            const int i = (p + 1) * B + w + eb[s2];
            if (eb[s2] >= 0 && i < m)
                at(i, i - w + eoff[s2]) = eu[s2] >= 0 ? stage[((p + 1) & 1) * B * NSD + eu[s2]] : 0.0;
        }
        if (loader) {
            stage[(p & 1) * B * NSD + t] = pf;
            pf = entering(p + 3, t);
        }
        lds_barrier();
    }
    if (bad) atomicOr(flags, F_BREAK_COARSE);
}

// The factor's rows as the one-wave solve reads them (see BandSolve): CF from
// L as for L D L^T, CG from U (the backward step k removes U_ik x_k).
__global__ void k_band_expand_ldu(int nc, const double *__restrict__ Lb, const double *__restrict__ Ub,
                                  const double *__restrict__ D, double *__restrict__ CF, double *__restrict__ CG,
                                  double *__restrict__ Dp)
{
    const int m = nc * nc, w = nc + 1, M = band_padded(m);
    const int l = threadIdx.x & 63;
    const int s = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (s >= M) return;
    const int q = s >> 6, r = s & 63;
    auto Lik = [&](int i, int k) -> double {
        return (i < m && k >= 0 && k < i && i - k <= w) ? Lb[(size_t)i * w + (k - i + w)] : 0.0;
    };
    auto Uik = [&](int i, int k) -> double {
        return (i >= 0 && k < m && i < k && k - i <= w) ? Ub[(size_t)i * w + (k - i - 1)] : 0.0;
    };
    const size_t o = (size_t)s * 64 + l;
    CF[o] = l > r ? Lik(64 * q + l, s) : Lik(64 * q + 64 + l, s);
    CG[o] = l < r ? Uik(64 * q + l, s) : (q >= 1 ? Uik(64 * q - 64 + l, s) : 0.0);
    if (l == 0) Dp[s] = s < m ? D[s] : 1.0;
}

// Partial sums of the squared residual of level 0 without storing it: the
// rows, threads, loop order and block reduction of k_sumsq_partial over the
// stored residual, and each r formed as k_ns_residual forms it, so the
// partial sums are the same to the bit.
__global__ __launch_bounds__(256) void k_ns_resid_sumsq(LevN L, double *__restrict__ part)
{
    double acc = 0.0;
    const int n = L.n;
    for (int j = 1 + blockIdx.x; j <= n; j += gridDim.x) {
        for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x) {
            const size_t p = (size_t)j * L.ld + i;
            double s = ns_offdiag(L, L.u, p);
            s -= L.A[E_O][p] * L.u[p];
            acc += s * s;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Sum of the np <= NPART_ROWS partial sums in order: the wave stages them in
// LDS (16 loads in flight per lane), then lane 0 adds them up from there.
__global__ __launch_bounds__(64) void k_ns_sum(const double *__restrict__ part, int np, double *__restrict__ out)
{
    static_assert(NPART_ROWS <= 16 * 64, "one round of loads stages the partials");
    __shared__ double sp[NPART_ROWS];
    const int lane = threadIdx.x;
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = lane + 64 * k < np ? part[lane + 64 * k] : 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (lane + 64 * k < np) sp[lane + 64 * k] = v[k];
    __syncthreads();
    if (lane != 0) return;
    double s = 0.0;
    for (int t = 0; t < np; ++t) s += sp[t];
    *out = s;
}

// Dense n x n <-> padded level interior.
__global__ void k_ns_pack(const double *__restrict__ src, int n, int ld, double *__restrict__ dst, bool in)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > n || j > n) return;
    const size_t p = (size_t)j * ld + i, t = (size_t)(j - 1) * n + (i - 1);
    if (in) dst[p] = src[t];
    else dst[t] = src[p];
}

}  // namespace

// ---------------------------------------------------------------- handle
struct bmg_ns {
    int n = 0, nlev = 0;
    bmg_options opt{};
    hipStream_t st = nullptr;
    char *ws = nullptr;
    LevN L[MAXL];
    Wts<double> P[MAXL], R[MAXL];
    double *Lb = nullptr, *Ub = nullptr, *Dd = nullptr;
    BandSolve band{};
    int *flags = nullptr;
    double *part = nullptr, *scal = nullptr, *hist = nullptr;
};

namespace {

const dim3 NB(32, 8);

// Workspace layout; with base == nullptr it only measures.
size_t ns_plan(bmg_ns *h, int n, const bmg_options &o, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + ALIGN - 1) & ~(ALIGN - 1);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const int nc0 = o.coarsest_n > 0 ? o.coarsest_n : 3;
    int nl = 0, ns[MAXL];
    for (int m = n; m >= nc0 && nl < MAXL; m = (m - 1) / 2) ns[nl++] = m;
    for (int l = 0; l < nl; ++l) {
        const int ld = pitch_of(ns[l]);
        const size_t pl = (size_t)(ns[l] + 2) * ld * sizeof(double);
        LevN L{};
        L.n = ns[l];
        L.ld = ld;
        for (int e = 0; e < NSD; ++e) L.A[e] = (double *)take(pl);
        L.u = (double *)take(pl);
        L.b = (double *)take(pl);
        L.r = (double *)take(pl);
        Wts<double> P{}, R{};
        if (l + 1 < nl) {
            const int ldc = pitch_of(ns[l + 1]);
            const size_t ps = (size_t)(ns[l + 1] + 2) * ldc;
            P = Wts<double>{(double *)take(8 * ps * sizeof(double)), ldc, ps};
            R = Wts<double>{(double *)take(8 * ps * sizeof(double)), ldc, ps};
        }
        if (h) {
            h->L[l] = L;
            h->P[l] = P;
            h->R[l] = R;
        }
    }
    const int cm = ns[nl - 1] * ns[nl - 1], cw = ns[nl - 1] + 1, cM = band_padded(cm);
    double *Lb = (double *)take((size_t)cm * cw * 8);
    double *Ub = (double *)take((size_t)cm * cw * 8);
    double *Dd = (double *)take((size_t)cm * 8);
    double *CF = (double *)take((size_t)cM * 64 * 8);
    double *CG = (double *)take((size_t)cM * 64 * 8);
    double *Dp = (double *)take((size_t)cM * 8);
    int *flags = (int *)take(64);
    double *part = (double *)take(NPART_ROWS * 8);
    double *scal = (double *)take(8 * 8);
    double *hist = (double *)take((size_t)(o.max_cycles + 1) * 8);
    if (h) {
        h->nlev = nl;
        h->Lb = Lb;
        h->Ub = Ub;
        h->Dd = Dd;
        h->band = BandSolve{CF, CG, Dp, cm, cM, ns[nl - 1]};
        h->flags = flags;
        h->part = part;
        h->scal = scal;
        h->hist = hist;
    }
    return (off + ALIGN - 1) & ~(ALIGN - 1);
}

bmg_status ns_check(int n, int kind, const bmg_options *o, bmg_options *op)
{
    if (!valid_n(n)) return fail(BMG_EINVAL, "n=%d is not 2^m-1 with 2 <= m <= 15", n);
    if (kind != 5 && kind != 9) return fail(BMG_EINVAL, "stencil kind %d is not 5 or 9", kind);
    bmg_default_options(op);
    if (o) *op = *o;
    if (op->nu1 < 0 || op->nu2 < 0 || op->nu1 + op->nu2 < 1 || op->max_cycles < 1)
        return fail(BMG_EINVAL, "bad cycle options");
    if (op->precision != BMG_FP64 || op->smoother != BMG_SMOOTH_POINT || op->interp != BMG_INTERP_BOXMG)
        return fail(BMG_EINVAL, "the nonsymmetric solver runs FP64 point relaxation with operator-induced weights");
    const int nc = op->coarsest_n > 0 ? op->coarsest_n : 3;
    if (!valid_n(nc) || nc > BAND_MAX_NC || nc > n)
        return fail(BMG_EINVAL, "coarsest_n=%d must be 2^k-1 in [3, min(%d, n)]", nc, BAND_MAX_NC);
    return BMG_OK;
}

Lev<double> as_lev(const LevN &L)
{
    Lev<double> v{};
    v.n = L.n;
    v.ld = L.ld;
    v.u = L.u;
    v.b = L.b;
    v.r = L.r;
    return v;
}

bmg_status ns_gs(bmg_ns *h, int l, int sweeps)
{
    const LevN &L = h->L[l];
    // colours 0, 1 (even rows), then 2, 3 (odd rows): rows of each parity
    const int rows[2] = {(L.n - 1) / 2, (L.n + 1) / 2};
    for (int s = 0; s < sweeps; ++s)
        for (int rp = 0; rp < 2; ++rp)
            hipLaunchKernelGGL(k_ns_gs_pair, dim3((rows[rp] + NS_PAIR_WAVES - 1) / NS_PAIR_WAVES),
                               dim3(64 * NS_PAIR_WAVES), 0, h->st, L, rp);
    LAUNCHCHK();
    return BMG_OK;
}

bmg_status ns_residual(bmg_ns *h, int l)
{
    const LevN &L = h->L[l];
    hipLaunchKernelGGL(k_ns_residual, grid2(L.n, L.n, NB), NB, 0, h->st, L);
    LAUNCHCHK();
    return BMG_OK;
}

bmg_status ns_restrict(bmg_ns *h, int l)
{
    const LevN &F = h->L[l];
    const Lev<double> Cl = as_lev(h->L[l + 1]);
    hipLaunchKernelGGL((k_restrict<double>), grid2(Cl.n, Cl.n, NB), NB, 0, h->st, (const double *)F.r, F.ld,
                       h->R[l], Cl, nullptr);
    LAUNCHCHK();
    return BMG_OK;
}

bmg_status ns_interp(bmg_ns *h, int l)
{
    const Lev<double> F = as_lev(h->L[l]);
    launch_interp_add<double>(F, h->P[l], (const double *)h->L[l + 1].u, nullptr, h->st);
    LAUNCHCHK();
    return BMG_OK;
}

bmg_status ns_coarse(bmg_ns *h)
{
    static bool attr = false;
    if (!attr) {
        HIPCHK(hipFuncSetAttribute((const void *)k_coarse_solve<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)band_solve_lds(band_padded(BAND_MAX_NC * BAND_MAX_NC))));
        attr = true;
    }
    const Lev<double> Cl = as_lev(h->L[h->nlev - 1]);
    hipLaunchKernelGGL((k_coarse_solve<double>), dim3(1), dim3(BAND_SOLVE_THREADS), band_solve_lds(h->band.M), h->st,
                       Cl, h->band, (size_t)0, nullptr, 0);
    LAUNCHCHK();
    return BMG_OK;
}

bmg_status ns_vcycle(bmg_ns *h, int l)
{
    if (l == h->nlev - 1) return ns_coarse(h);
    TRY(ns_gs(h, l, h->opt.nu1));
    TRY(ns_residual(h, l));
    TRY(ns_restrict(h, l));   // also zeroes u on level l + 1
    TRY(ns_vcycle(h, l + 1));
    TRY(ns_interp(h, l));
    return ns_gs(h, l, h->opt.nu2);
}

// sum of squares of level 0's residual into scal[slot] (the value of
// ns_residual then ns_sumsq of r, without writing r)
bmg_status ns_resnorm(bmg_ns *h, int slot)
{
    const int nb = std::min(NPART_ROWS, h->L[0].n);
    hipLaunchKernelGGL(k_ns_resid_sumsq, dim3(nb), dim3(256), 0, h->st, h->L[0], h->part);
    hipLaunchKernelGGL(k_ns_sum, dim3(1), dim3(64), 0, h->st, (const double *)h->part, nb, h->scal + slot);
    LAUNCHCHK();
    return BMG_OK;
}

// sum of squares of level 0's interior of x into scal[slot]
bmg_status ns_sumsq(bmg_ns *h, const double *x, int slot)
{
    const Lev<double> L = as_lev(h->L[0]);
    const int nb = std::min(NPART_ROWS, L.n);
    hipLaunchKernelGGL((k_sumsq_partial<double, false, false>), dim3(nb), dim3(256), 0, h->st, L, x, h->part,
                       nullptr);
    hipLaunchKernelGGL(k_ns_sum, dim3(1), dim3(64), 0, h->st, (const double *)h->part, nb, h->scal + slot);
    LAUNCHCHK();
    return BMG_OK;
}

}  // namespace

extern "C" {

bmg_status bmg_ns_workspace_bytes(int n, int kind, const bmg_options *o, size_t *bytes)
{
    if (!bytes) return fail(BMG_EINVAL, "NULL argument");
    bmg_options op;
    TRY(ns_check(n, kind, o, &op));
    *bytes = ns_plan(nullptr, n, op, nullptr);
    return BMG_OK;
}

bmg_status bmg_ns_setup(bmg_ns **out, const double *stencil, int n, int kind, const bmg_options *o, void *workspace,
                        size_t ws_bytes, bmg_stream stream)
{
    if (!out || !stencil) return fail(BMG_EINVAL, "NULL argument");
    *out = nullptr;
    bmg_options op;
    TRY(ns_check(n, kind, o, &op));
    const size_t need = ns_plan(nullptr, n, op, nullptr);
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace & (ALIGN - 1)))
        return fail(BMG_EWORKSPACE, "workspace %p of %zu bytes; need %zu bytes, 256-byte aligned", workspace,
                    ws_bytes, need);
    bmg_ns *h = new bmg_ns();
    h->n = n;
    h->opt = op;
    h->st = (hipStream_t)stream;
    h->ws = (char *)workspace;
    ns_plan(h, n, op, h->ws);
    auto bail = [&](bmg_status s) {
        delete h;
        return s;
    };
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute((const void *)k_band_ldu_factor, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)ns_band_lds()) != hipSuccess)
            return bail(fail(BMG_EDEVICE, "LDS attribute of the band factor"));
        attr = true;
    }
    if (hipMemsetAsync(h->ws, 0, need, h->st) != hipSuccess) return bail(fail(BMG_EDEVICE, "workspace clear failed"));
    hipLaunchKernelGGL(k_ns_import, grid2(n, n, NB), NB, 0, h->st, stencil, kind, h->L[0], h->flags);
    for (int l = 0; l + 1 < h->nlev; ++l) {
        const int nc = h->L[l + 1].n;
        for (int tr = 0; tr < 2; ++tr) {
            const Wts<double> &C = tr ? h->R[l] : h->P[l];
            hipLaunchKernelGGL(k_ns_weights_edges, grid2(nc + 1, nc + 1, NB), NB, 0, h->st, h->L[l], C, nc, tr != 0,
                               h->flags);
            hipLaunchKernelGGL(k_ns_weights_corners, grid2(nc + 1, nc + 1, NB), NB, 0, h->st, h->L[l], C, nc,
                               tr != 0, h->flags);
        }
        hipLaunchKernelGGL(k_ns_rap, grid2(nc, nc, NB), NB, 0, h->st, h->L[l], h->P[l], h->R[l], h->L[l + 1]);
    }
    hipLaunchKernelGGL(k_band_ldu_factor, dim3(1), dim3(NSB_THREADS), ns_band_lds(), h->st, h->L[h->nlev - 1], h->Lb,
                       h->Ub, h->Dd, h->flags);
    hipLaunchKernelGGL(k_band_expand_ldu, dim3(h->band.M / 4), dim3(256), 0, h->st, h->band.nc,
                       (const double *)h->Lb, (const double *)h->Ub, (const double *)h->Dd, (double *)h->band.CF,
                       (double *)h->band.CG, (double *)h->band.Dp);
    if (hipGetLastError() != hipSuccess) return bail(fail(BMG_EDEVICE, "set-up kernel launch failed"));
    int flags = 0;
    if (hipMemcpyAsync(&flags, h->flags, sizeof flags, hipMemcpyDeviceToHost, h->st) != hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess)
        return bail(fail(BMG_EDEVICE, "reading the set-up flags failed"));
    if (flags & (F_NONFINITE | F_DIAG | F_BOUNDARY))
        return bail(fail(BMG_EINVAL, "stencil rejected:%s%s%s", (flags & F_NONFINITE) ? " non-finite entry" : "",
                         (flags & F_DIAG) ? " centre <= 0" : "", (flags & F_BOUNDARY) ? " coupling to the boundary" : ""));
    if (flags & (F_BREAK_INTERP | F_BREAK_COARSE))
        return bail(fail(BMG_EBREAKDOWN, "%s", (flags & F_BREAK_INTERP) ? "interpolation denominator <= 0"
                                                                        : "coarsest pivot <= 0"));
    *out = h;
    return BMG_OK;
}

bmg_status bmg_ns_solve(bmg_ns *h, const double *rhs, double *x, double tol, bmg_info *info)
{
    if (!h || !rhs || !x) return fail(BMG_EINVAL, "NULL argument");
    if (!(tol >= 0.0)) return fail(BMG_EINVAL, "tol must be >= 0");
    LevN &L = h->L[0];
    const int n = L.n;
    const dim3 g = grid2(n, n, NB);
    hipLaunchKernelGGL(k_ns_pack, g, NB, 0, h->st, rhs, n, L.ld, L.b, true);
    hipLaunchKernelGGL(k_ns_pack, g, NB, 0, h->st, (const double *)x, n, L.ld, L.u, true);
    LAUNCHCHK();
    TRY(ns_sumsq(h, L.b, 0));
    double nb2 = 0.0;
    HIPCHK(hipMemcpyAsync(&nb2, h->scal, sizeof nb2, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    int k = 0;
    double rho = 0.0, first = 0.0;
    if (nb2 == 0.0) {
        HIPCHK(hipMemsetAsync(x, 0, (size_t)n * n * sizeof(double), h->st));
        HIPCHK(hipStreamSynchronize(h->st));
    } else {
        const double nb = sqrt(nb2);
        while (k < h->opt.max_cycles) {
            TRY(ns_vcycle(h, 0));
            TRY(ns_resnorm(h, 1));
            double rr = 0.0;
            HIPCHK(hipMemcpyAsync(&rr, h->scal + 1, sizeof rr, hipMemcpyDeviceToHost, h->st));
            HIPCHK(hipStreamSynchronize(h->st));
            rho = sqrt(rr) / nb;
            if (k == 0) first = rho;
            if (info && info->history) info->history[k] = rho;
            ++k;
            if (!(rho > tol)) break;
            if (!isfinite(rho)) break;
        }
        hipLaunchKernelGGL(k_ns_pack, g, NB, 0, h->st, (const double *)L.u, n, L.ld, x, false);
        LAUNCHCHK();
        HIPCHK(hipStreamSynchronize(h->st));
    }
    if (info) {
        info->cycles = k;
        info->rel_res = rho;
        info->rho = k > 1 ? pow(rho / first, 1.0 / (k - 1)) : 0.0;
        info->floor_est = 0.0;
        info->t_setup_ms = 0.0;
        info->t_solve_ms = 0.0;
        info->interp_used = BMG_INTERP_BOXMG;
        info->learned_levels_used = 0;
    }
    if (!isfinite(rho)) return fail(BMG_EDIVERGED, "residual is not finite after %d cycles", k);
    if (rho > tol) return fail(BMG_ENOCONV, "relative residual %.3e > tol %.3e after %d cycles", rho, tol, k);
    return BMG_OK;
}

bmg_status bmg_ns_destroy(bmg_ns *h)
{
    delete h;
    return BMG_OK;
}

bmg_status bmg_ns_num_levels(const bmg_ns *h, int *nlev)
{
    if (!h || !nlev) return fail(BMG_EINVAL, "NULL argument");
    *nlev = h->nlev;
    return BMG_OK;
}

bmg_status bmg_ns_level_n(const bmg_ns *h, int level, int *n)
{
    if (!h || !n) return fail(BMG_EINVAL, "NULL argument");
    if (level < 0 || level >= h->nlev) return fail(BMG_EINVAL, "level %d out of range", level);
    *n = h->L[level].n;
    return BMG_OK;
}

// Field ids: 0..8 stencil planes, 9 P's weights, 10 R's weights, 11 u, 12 b,
// 13 r (padded (n+2)^2 or 8 planes of (nc+2)^2), 14 the coarsest factor
// (L band m w, U band m w, D m).
static bmg_status ns_locate(bmg_ns *h, int level, int field, double **ptr, size_t *pitch, size_t *rows, size_t *width,
                            size_t *nplanes, size_t *pstride)
{
    if (!h) return fail(BMG_EINVAL, "NULL handle");
    *nplanes = 1;
    *pstride = 0;
    if (field == 14) {
        const size_t m = h->band.m, w = h->band.nc + 1, cnt = 2 * m * w + m;
        // Lb, Ub and D are consecutive in the workspace only up to alignment: copied piecewise by the caller
        *ptr = h->Lb;
        *pitch = cnt;
        *rows = 1;
        *width = cnt;
        return BMG_OK;
    }
    if (level < 0 || level >= h->nlev) return fail(BMG_EINVAL, "level %d out of range", level);
    const LevN &L = h->L[level];
    if (field >= 0 && field < NSD) {
        *ptr = L.A[field];
    } else if (field == 9 || field == 10) {
        if (level + 1 >= h->nlev) return fail(BMG_EINVAL, "no weights below the coarsest level");
        const Wts<double> &C = field == 9 ? h->P[level] : h->R[level];
        *ptr = C.p;
        *pitch = C.ld;
        *rows = h->L[level + 1].n + 2;
        *width = h->L[level + 1].n + 2;
        *nplanes = 8;
        *pstride = C.ps;
        return BMG_OK;
    } else if (field == 11) {
        *ptr = L.u;
    } else if (field == 12) {
        *ptr = L.b;
    } else if (field == 13) {
        *ptr = L.r;
    } else {
        return fail(BMG_EINVAL, "unknown field %d", field);
    }
    *pitch = L.ld;
    *rows = L.n + 2;
    *width = L.n + 2;
    return BMG_OK;
}

bmg_status bmg_ns_export(bmg_ns *h, int level, int field, double *dst)
{
    if (!dst) return fail(BMG_EINVAL, "NULL argument");
    double *p;
    size_t pitch, rows, width, np, ps;
    TRY(ns_locate(h, level, field, &p, &pitch, &rows, &width, &np, &ps));
    if (field == 14) {
        const size_t m = h->band.m, w = h->band.nc + 1;
        HIPCHK(hipMemcpyAsync(dst, h->Lb, m * w * 8, hipMemcpyDeviceToDevice, h->st));
        HIPCHK(hipMemcpyAsync(dst + m * w, h->Ub, m * w * 8, hipMemcpyDeviceToDevice, h->st));
        HIPCHK(hipMemcpyAsync(dst + 2 * m * w, h->Dd, m * 8, hipMemcpyDeviceToDevice, h->st));
    } else {
        for (size_t k = 0; k < np; ++k)
            HIPCHK(hipMemcpy2DAsync(dst + k * rows * width, width * 8, p + k * ps, pitch * 8, width * 8, rows,
                                    hipMemcpyDeviceToDevice, h->st));
    }
    HIPCHK(hipStreamSynchronize(h->st));
    return BMG_OK;
}

bmg_status bmg_ns_import(bmg_ns *h, int level, int field, const double *src)
{
    if (!src) return fail(BMG_EINVAL, "NULL argument");
    if (field < 11 || field > 13) return fail(BMG_EINVAL, "only u, b and r can be imported");
    double *p;
    size_t pitch, rows, width, np, ps;
    TRY(ns_locate(h, level, field, &p, &pitch, &rows, &width, &np, &ps));
    HIPCHK(hipMemcpy2DAsync(p, pitch * 8, src, width * 8, width * 8, rows, hipMemcpyDeviceToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return BMG_OK;
}

// One step on level l's arrays: 0 = arg sweeps, 1 = residual, 2 = restriction
// into b_{l+1} (u_{l+1} zeroed), 3 = u += P u_{l+1}, 4 = coarsest solve.
bmg_status bmg_ns_step(bmg_ns *h, int level, int step, int arg)
{
    if (!h) return fail(BMG_EINVAL, "NULL handle");
    if (level < 0 || level >= h->nlev) return fail(BMG_EINVAL, "level %d out of range", level);
    const bool coarse = level == h->nlev - 1;
    switch (step) {
    case 0: TRY(ns_gs(h, level, arg)); break;
    case 1: TRY(ns_residual(h, level)); break;
    case 2: if (coarse) return fail(BMG_EINVAL, "no level below"); TRY(ns_restrict(h, level)); break;
    case 3: if (coarse) return fail(BMG_EINVAL, "no level below"); TRY(ns_interp(h, level)); break;
    case 4: if (!coarse) return fail(BMG_EINVAL, "the direct solve runs on the coarsest level"); TRY(ns_coarse(h)); break;
    default: return fail(BMG_EINVAL, "unknown step %d", step);
    }
    HIPCHK(hipStreamSynchronize(h->st));
    return BMG_OK;
}

}  // extern "C"
