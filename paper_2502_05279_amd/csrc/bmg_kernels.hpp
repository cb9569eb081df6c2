// HIP kernels (gfx950) of the black-box multigrid V-cycle: discretisation,
// set-up (operator-induced interpolation, Galerkin coarse operators, coarsest
// LDL^T factor) and the per-level cycle steps (four-colour Gauss-Seidel,
// residual, restriction, interpolation, norms).
//
// All floating-point expressions are written in one fixed order and the
// library is compiled with -ffp-contract=off, so every point's result is the
// correctly rounded value of that expression sequence (IEEE division
// included); schedules that respect the colour dependencies produce the same
// bits.
//
// Level arrays are (n+2) rows of `ld` elements, row j (north) after row j-1,
// element (i,j) at j*ld + i; rows/columns 0 and n+1 are the Dirichlet ring and
// hold zeros.  Stencils are symmetric-compact: O, W, S on every level plus SW,
// NW on nine-point levels; the east / north / north-east / south-east entries
// of point p are W(p+1), S(p+ld), SW(p+ld+1), NW(p+1-ld).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmg {

template <typename T>
struct Lev {
    int n;   // interior points per side
    int ld;  // row pitch (elements)
    T *u, *b, *r;
    T *O, *W, *S, *SW, *NW;  // SW, NW null on five-point levels
};

// Weights between a fine level and the next coarser one: 8 planes
// (LNE, LA, LNW, LR, LL, LSE, LB, LSW) of the coarse level's shape.
template <typename T>
struct Wts {
    T *p;
    int ld;       // coarse row pitch
    size_t ps;    // plane stride (elements)
    __device__ __forceinline__ T at(int plane, size_t c) const { return p[plane * ps + c]; }
};

enum : int { LNE = 0, LA = 1, LNW = 2, LR = 3, LL = 4, LSE = 5, LB = 6, LSW = 7 };

// validation / breakdown flag bits
enum : int {
    F_NONFINITE = 1, F_DIAG = 2, F_BOUNDARY = 4, F_ASYM = 8,
    F_BREAK_INTERP = 16, F_BREAK_COARSE = 32, F_BREAK_LINE = 64
};

__device__ __forceinline__ bool stopped(const int *stop) { return stop && *stop; }

// --------------------------------------------------------------- discretise
// Vertex-centred five-point operator of -div(k grad u) = f, cell-constant k:
// coupling = -(mean of the two cells sharing the grid edge), centre = minus the
// sum of the four couplings (before the boundary couplings are zeroed),
// right-hand side h^2 f.  Output [n][n][5] = S, W, O, E, N.
static __global__ void k_discretize(const double *__restrict__ k, const double *__restrict__ f,
                             int n, double h2, double *__restrict__ st,
                             double *__restrict__ rhs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int j = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (i > n || j > n) return;
    const size_t lk = (size_t)n + 1;
    const double kSW = k[(size_t)(j - 1) * lk + (i - 1)];
    const double kSE = k[(size_t)(j - 1) * lk + i];
    const double kNW = k[(size_t)j * lk + (i - 1)];
    const double kNE = k[(size_t)j * lk + i];
    double aW = -0.5 * (kSW + kNW);
    double aE = -0.5 * (kSE + kNE);
    double aS = -0.5 * (kSW + kSE);
    double aN = -0.5 * (kNW + kNE);
    const double aO = -(((aW + aE) + aS) + aN);
    if (i == 1) aW = 0.0;
    if (i == n) aE = 0.0;
    if (j == 1) aS = 0.0;
    if (j == n) aN = 0.0;
    const size_t q = (size_t)(j - 1) * n + (i - 1);
    double *o = st + q * 5;
    o[0] = aS; o[1] = aW; o[2] = aO; o[3] = aE; o[4] = aN;
    rhs[q] = h2 * f[q];
}

// ------------------------------------------------------------ import stencil
__device__ __forceinline__ bool asym(double a, double b)
{
    const double d = fabs(a - b), m = fmax(fabs(a), fabs(b));
    return !(d <= 1e-14 * m);
}

// [n][n][K] user stencil -> compact level-0 planes, with validation.
static __global__ void k_import_stencil(const double *__restrict__ st, int K, Lev<double> L,
                                 int *__restrict__ flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int j = blockIdx.y * blockDim.y + threadIdx.y + 1;
    const int n = L.n;
    if (i > n || j > n) return;
    const size_t q = ((size_t)(j - 1) * n + (i - 1)) * K;
    const size_t p = (size_t)j * L.ld + i;
    int bad = 0;
    double e[9];
    // e[] in the order SW, S, SE, W, O, E, NW, N, NE
    if (K == 5) {
        e[0] = 0.0; e[1] = st[q + 0]; e[2] = 0.0; e[3] = st[q + 1]; e[4] = st[q + 2];
        e[5] = st[q + 3]; e[6] = 0.0; e[7] = st[q + 4]; e[8] = 0.0;
    } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) e[t] = st[q + t];
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
        if (!isfinite(e[t])) bad |= F_NONFINITE;
    if (!(e[4] > 0.0)) bad |= F_DIAG;
    if (i == 1 && (e[0] != 0.0 || e[3] != 0.0 || e[6] != 0.0)) bad |= F_BOUNDARY;
    if (i == n && (e[2] != 0.0 || e[5] != 0.0 || e[8] != 0.0)) bad |= F_BOUNDARY;
    if (j == 1 && (e[0] != 0.0 || e[1] != 0.0 || e[2] != 0.0)) bad |= F_BOUNDARY;
    if (j == n && (e[6] != 0.0 || e[7] != 0.0 || e[8] != 0.0)) bad |= F_BOUNDARY;
    // symmetry against the neighbours' west / south / south-west / north-west
    if (i < n) {
        const size_t qe = q + K;
        if (asym(e[5], K == 5 ? st[qe + 1] : st[qe + 3])) bad |= F_ASYM;
    }
    if (j < n) {
        const size_t qn = q + (size_t)n * K;
        if (asym(e[7], K == 5 ? st[qn + 0] : st[qn + 1])) bad |= F_ASYM;
    }
    if (K == 9) {
        if (i < n && j < n && asym(e[8], st[q + ((size_t)n + 1) * K + 0])) bad |= F_ASYM;
        if (i < n && j > 1 && asym(e[2], st[q - ((size_t)n - 1) * K + 6])) bad |= F_ASYM;
    }
    L.O[p] = e[4];
    L.W[p] = e[3];
    L.S[p] = e[1];
    if (L.SW) {
        L.SW[p] = e[0];
        L.NW[p] = e[6];
    }
    if (bad) atomicOr(flags, bad);
}

// ------------------------------------------------- interpolation weights
// Row p of a compact stencil: SW, S, SE, W, O, E, NW, N, NE (a five-point
// stencil has no SW and NW planes: its corners are zero).
template <bool NINE>
__device__ __forceinline__ void row_of(const Lev<double> &L, size_t p, double a[9])
{
    const size_t ld = L.ld;
    a[0] = NINE ? L.SW[p] : 0.0;
    a[1] = L.S[p];
    a[2] = NINE ? L.NW[p + 1 - ld] : 0.0;
    a[3] = L.W[p];
    a[4] = L.O[p];
    a[5] = L.W[p + 1];
    a[6] = NINE ? L.NW[p] : 0.0;
    a[7] = L.S[p + ld];
    a[8] = NINE ? L.SW[p + ld + 1] : 0.0;
}

// Positive off-diagonals moved onto the diagonal (SW,S,SE,W,E,NW,N,NE order).
__device__ __forceinline__ void lump_row(double a[9])
{
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        if (e == 4) continue;
        if (a[e] > 0.0) {
            a[4] = a[4] + a[e];
            a[e] = 0.0;
        }
    }
}

// Edge weights: x-edge X(I,J) = (2I-1, 2J) for I <= nc+1, J <= nc collapses the
// lumped stencil along y; y-edge Y(I,J) = (2I, 2J-1) for I <= nc, J <= nc+1
// collapses along x.
template <bool NINE>
static __global__ void k_weights_edges(Lev<double> F, Wts<double> C, int nc, int *__restrict__ flags)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int J = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (I > nc + 1 || J > nc + 1) return;
    const size_t c = (size_t)J * C.ld + I;
    const size_t ld = F.ld;
    int bad = 0;
    double a[9];
    if (J <= nc) {
        row_of<NINE>(F, (size_t)(2 * J) * ld + (2 * I - 1), a);
        lump_row(a);
        const double D = (a[4] + a[7]) + a[1];
        if (!(D > 0.0)) bad = F_BREAK_INTERP;
        C.p[LL * C.ps + c] = -((a[3] + a[6]) + a[0]) / D;
        C.p[LR * C.ps + c] = -((a[5] + a[8]) + a[2]) / D;
    }
    if (I <= nc) {
        row_of<NINE>(F, (size_t)(2 * J - 1) * ld + (2 * I), a);
        lump_row(a);
        const double D = (a[4] + a[3]) + a[5];
        if (!(D > 0.0)) bad = F_BREAK_INTERP;
        C.p[LB * C.ps + c] = -((a[1] + a[0]) + a[2]) / D;
        C.p[LA * C.ps + c] = -((a[7] + a[6]) + a[8]) / D;
    }
    if (bad) atomicOr(flags, bad);
}

// Cell-centre weights at Z(I,J) = (2I-1, 2J-1), I, J <= nc+1, from the lumped
// stencil and the neighbouring edge weights.
template <bool NINE>
static __global__ void k_weights_corners(Lev<double> F, Wts<double> C, int nc, int *__restrict__ flags)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int J = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (I > nc + 1 || J > nc + 1) return;
    const size_t c = (size_t)J * C.ld + I;
    const size_t cs = c - C.ld, cw = c - 1;
    double a[9];
    row_of<NINE>(F, (size_t)(2 * J - 1) * F.ld + (2 * I - 1), a);
    lump_row(a);
    if (!(a[4] > 0.0)) atomicOr(flags, F_BREAK_INTERP);
    const double lr = C.at(LR, c), ll = C.at(LL, c), la = C.at(LA, c), lb = C.at(LB, c);
    const double lr_s = C.at(LR, cs), ll_s = C.at(LL, cs);
    const double la_w = C.at(LA, cw), lb_w = C.at(LB, cw);
    C.p[LNE * C.ps + c] = -((a[8] + a[7] * lr) + a[5] * la) / a[4];
    C.p[LNW * C.ps + c] = -((a[6] + a[7] * ll) + a[3] * la_w) / a[4];
    C.p[LSE * C.ps + c] = -((a[2] + a[1] * lr_s) + a[5] * lb) / a[4];
    C.p[LSW * C.ps + c] = -((a[0] + a[1] * ll_s) + a[3] * lb_w) / a[4];
}

// --------------------------------------------------------- Galerkin RAP
// Weight of coarse basis function K = (KI,KJ) at fine point 2K + (di,dj).
__device__ __forceinline__ double basis_weight(const Wts<double> &C, int KI, int KJ, int di, int dj)
{
    const size_t c = (size_t)KJ * C.ld + KI;
    if (dj == 0) {
        if (di == 0) return 1.0;
        return di < 0 ? C.at(LR, c) : C.at(LL, c + 1);
    }
    if (dj < 0) {
        if (di == 0) return C.at(LA, c);
        return di < 0 ? C.at(LNE, c) : C.at(LNW, c + 1);
    }
    if (di == 0) return C.at(LB, c + C.ld);
    return di < 0 ? C.at(LSE, c + C.ld) : C.at(LSW, c + C.ld + 1);
}

// A_c(I,J;d) = sum_p P(p;IJ) sum_q A(p,q) P(q;IJ+d), d = O, W, S, SW, NW, p over
// the fine 3x3 patch of (2I,2J) (rows south to north, west to east inside a
// row), q over p's neighbours SW..NE inside the support of basis IJ+d; both
// sums start from zero.  Couplings to ring coarse points are zero: their sums
// are formed with the weights of the nearest interior point (so every load
// is in range and none waits behind a branch) and then replaced by zero.
template <bool NINE>
static __global__ __launch_bounds__(128) void k_rap(Lev<double> F, Wts<double> C, Lev<double> Cl)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int J = blockIdx.y * blockDim.y + threadIdx.y + 1;
    const int nc = Cl.n;
    if (I > nc || J > nc) return;
    constexpr int offI[5] = {0, -1, 0, -1, -1};
    constexpr int offJ[5] = {0, 0, -1, -1, 1};
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    bool live[5];
    int KI[5], KJ[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        const int ki = I + offI[d], kj = J + offJ[d];
        live[d] = ki >= 1 && kj >= 1 && kj <= nc;
        KI[d] = ki < 1 ? 1 : ki;
        KJ[d] = kj < 1 ? 1 : kj > nc ? nc : kj;
    }
#pragma unroll
    for (int jj = -1; jj <= 1; ++jj) {
#pragma unroll
        for (int ii = -1; ii <= 1; ++ii) {
            const int pi = 2 * I + ii, pj = 2 * J + jj;
            double a[9];
            row_of<NINE>(F, (size_t)pj * F.ld + pi, a);
            const double wp = basis_weight(C, I, J, ii, jj);
#pragma unroll
            for (int d = 0; d < 5; ++d) {
                double t = 0.0;
#pragma unroll
                for (int e = 0; e < 9; ++e) {
                    // q - 2(IJ+d), the same for the clamped point's support
                    const int di = ii + (e % 3) - 1 - 2 * offI[d], dj = jj + (e / 3) - 1 - 2 * offJ[d];
                    if (di < -1 || di > 1 || dj < -1 || dj > 1) continue;
                    t = t + a[e] * basis_weight(C, KI[d], KJ[d], di, dj);
                }
                acc[d] = acc[d] + wp * t;
            }
        }
    }
    const size_t c = (size_t)J * Cl.ld + I;
    Cl.O[c] = acc[0];
    Cl.W[c] = live[1] ? acc[1] : 0.0;
    Cl.S[c] = live[2] ? acc[2] : 0.0;
    Cl.SW[c] = live[3] ? acc[3] : 0.0;
    Cl.NW[c] = live[4] ? acc[4] : 0.0;
}

// The set-up kernels of one level pair, for a five- or nine-point fine stencil.
static inline void launch_weights(const Lev<double> &F, const Wts<double> &C, int nc, int *flags, dim3 grid,
                                  dim3 blk, hipStream_t st)
{
    if (F.SW) {
        hipLaunchKernelGGL(k_weights_edges<true>, grid, blk, 0, st, F, C, nc, flags);
        hipLaunchKernelGGL(k_weights_corners<true>, grid, blk, 0, st, F, C, nc, flags);
    } else {
        hipLaunchKernelGGL(k_weights_edges<false>, grid, blk, 0, st, F, C, nc, flags);
        hipLaunchKernelGGL(k_weights_corners<false>, grid, blk, 0, st, F, C, nc, flags);
    }
}

static inline void launch_rap(const Lev<double> &F, const Wts<double> &C, const Lev<double> &Cl, hipStream_t st)
{
    const dim3 blk(32, 4), grid((Cl.n + 31) / 32, (Cl.n + 3) / 4);
    if (F.SW)
        hipLaunchKernelGGL(k_rap<true>, grid, blk, 0, st, F, C, Cl);
    else
        hipLaunchKernelGGL(k_rap<false>, grid, blk, 0, st, F, C, Cl);
}

// ------------------------------------------------ coarsest level: band LDL^T
// The coarsest level (nc points per side, 3 <= nc <= 63) is solved directly.
// Its unknowns in lexicographic order k = (i-1) + nc (j-1) give a band matrix
// of half-bandwidth w = nc + 1 <= 64, whose square-root-free Cholesky factor
// L D L^T stays inside the band.  Set-up keeps
//   Lb[i w + (k - i + w)] = L_ik  (k = i-w .. i-1, zero for k < 0), D[i];
// and, for the solve, the same entries rearranged by the lane that uses them
// (BandSolve below).
constexpr int BAND_MAX_NC = 63;

// A(i, i - d) of the coarsest level's matrix, d = 0 .. w, from its compact
// stencil: d = 1 W, nc - 1 SE (the NW entry of the point below-right), nc S,
// nc + 1 SW; couplings to points outside the grid are zero.
__device__ inline double band_entry(const Lev<double> &L, int i, int d)
{
    const int nc = L.n;
    const int ii = i % nc + 1, jj = i / nc + 1;
    const size_t p = (size_t)jj * L.ld + ii;
    if (d == 0) return L.O[p];
    if (d == 1) return ii > 1 ? L.W[p] : 0.0;
    if (d == nc - 1) return (ii < nc && jj > 1 && L.NW) ? L.NW[p + 1 - L.ld] : 0.0;
    if (d == nc) return jj > 1 ? L.S[p] : 0.0;
    if (d == nc + 1) return (ii > 1 && jj > 1 && L.SW) ? L.SW[p] : 0.0;
    return 0.0;
}

// A workgroup barrier that orders LDS only: loads from global memory stay in
// flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// v of lane `lane`, on every lane.
__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The factor in one workgroup, in right-looking form by panels of
// BAND_PANEL columns.  Once column k is final (D_k = a_kk, L_ik = a_ik / D_k,
// v_j = L_jk D_k), every entry of the trailing window takes its term,
// a_ij <- a_ij - L_ik v_j (k < j <= i <= k + w).  An entry thus receives its
// terms in order of increasing k, each the same product of the same operands
// as in the column-by-column sums of the definition
//   D_j = A_jj - sum_k L_jk v_k,  L_ij = (A_ij - sum_k L_ik v_k) / D_j,
// so the factor is the same to the bit.  A panel's columns are finished by
// wave 0 alone in registers, one after the other, together with the terms
// they give to the panel's own later columns (each lane holds two rows of
// the panel; the diagonal and the v values come from their rows' lanes by
// readlane); then every thread applies the panel's terms, in column order,
// to its entries of the trailing triangle and writes the panel's L and D to
// memory: two barriers per panel instead of two per column.  One wave's
// column chain is what the factor waits on, so that part is straight-line
// code with one division per lane and column and no stores to memory (at
// 63^2: 2.04 ms; 2.81 ms with predicated updates and the stores in wave 0,
// 2.92 ms by columns).  The window's rows live in an LDS ring (row i,
// column j at slot i mod RR, offset j - i + w); the B rows a panel adds to the
// window enter during the previous panel's trailing update, their entries of
// A requested from memory two panels ahead (registers, then a staging
// buffer), so no panel waits on memory.
constexpr int BAND_FACTOR_THREADS = 1024;
constexpr int BAND_NNZ = 5;   // lower-band entries of a row of A: distances 0, 1, nc - 1, nc, nc + 1
#ifndef BMG_BAND_PANEL
#define BMG_BAND_PANEL 8
#endif
constexpr int BAND_PANEL = BMG_BAND_PANEL;
static_assert(BAND_PANEL * (BAND_MAX_NC + 2) <= BAND_FACTOR_THREADS && BAND_PANEL <= 64,
              "the rows a panel adds take one thread per entry, and wave 0 holds the panel's rows");

__device__ inline int band_nz_dist(int e, int nc) { return e == 0 ? 0 : e == 1 ? 1 : e == 2 ? nc - 1 : e == 3 ? nc : nc + 1; }

static __global__ __launch_bounds__(BAND_FACTOR_THREADS) void k_band_factor(Lev<double> L, double *__restrict__ Lb,
                                                                             double *__restrict__ D,
                                                                             int *__restrict__ flags)
{
    constexpr int B = BAND_PANEL, RW = BAND_MAX_NC + 2, RR = BAND_MAX_NC + 1 + B;
    __shared__ double ring[RR * RW];
    __shared__ double Lp[B][RW], vp[B][RW];           // the panel's columns: L(k + d, k), v at offset d
    __shared__ double stage[2][B * BAND_NNZ];
    __shared__ double Dpan[B];
    const int nc = L.n, m = nc * nc, w = nc + 1, t = threadIdx.x;
    const int npanel = (m + B - 1) / B;
    auto at = [&](int i, int j) -> double & { return ring[(i % RR) * RW + (j - i + w)]; };
    // the rows panel q adds to the window: q B + w .. q B + w + B - 1; entry u
    // of its staging buffer is row q B + w + u / NNZ at distance nz(u % NNZ)
    auto entering = [&](int q, int u) -> double {
        const int i = q * B + w + u / BAND_NNZ;
        return i < m ? band_entry(L, i, band_nz_dist(u % BAND_NNZ, nc)) : 0.0;
    };
    // rows 0 .. w + B - 1 of A (the window of panel 0)
    for (int e = t; e < (w + B) * (w + 1); e += blockDim.x) {
        const int i = e / (w + 1), off = e % (w + 1), j = i - w + off;
        if (i < m) at(i, j) = j >= 0 ? band_entry(L, i, i - j) : 0.0;
    }
    const bool loader = t < B * BAND_NNZ;
    if (loader) stage[1] [t] = entering(1, t);
    double pf = loader ? entering(2, t) : 0.0;        // panel 2's rows, in flight
    // this thread's entries of the trailing triangle, e = t + s * blockDim.x
    const int ntri = w * (w + 1) / 2;
    int di[3], dj[3];
#pragma unroll
    for (int s2 = 0; s2 < 3; ++s2) {
        const int e = t + s2 * BAND_FACTOR_THREADS;
        int d = (int)((1.0f + sqrtf(8.0f * (float)e + 1.0f)) * 0.5f);
        while (d > 1 && d * (d - 1) / 2 > e) --d;
        while ((d + 1) * d / 2 <= e) ++d;
        di[s2] = e < ntri ? d : 0;
        dj[s2] = e - d * (d - 1) / 2 + 1;
    }
    // this thread's entry of the rows entering the window: row b, offset off
    const int eb = t / (w + 1), eoff = t % (w + 1);
    const bool enters = t < B * (w + 1);
    int eu = -1;   // its index in the staging buffer (-1: a zero of the band)
    if (enters) {
#pragma unroll
        for (int e = 0; e < BAND_NNZ; ++e)
            if (w - eoff == band_nz_dist(e, nc)) eu = eb * BAND_NNZ + e;
    }
    int bad = 0;
    lds_barrier();
    for (int p = 0; p < npanel; ++p) {
        const int k0 = p * B;
        if (t < 64) {
            // wave 0: the panel's columns, in registers.  Lane l holds the
            // panel entries of rows k0 + l and k0 + 64 + l.  The band rows
            // below the diagonal of column k = k0 + b are k + 1 .. k + 64:
            // the first row of lanes l > b and the second row of lanes
            // l <= b, so every lane divides once per column.  The diagonal
            // and the v of a later panel column come from the lane of its
            // row.  A row outside a column's band holds zeros there, and
            // rows past the matrix act as rows of the identity (D = 1, no
            // terms), so the work is the same straight-line code for every
            // panel; a lane's first row takes terms in every later panel
            // column (those right of its diagonal are never read again),
            // its second row only once it is the lane's row of the column
            const int r0 = k0 + t, r1 = k0 + 64 + t;
            double a0[B], a1[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int k = k0 + b;
                a0[b] = r0 >= m ? (r0 == k ? 1.0 : 0.0) : (r0 >= k && r0 - k <= w) ? at(r0, k) : 0.0;
                a1[b] = (r1 < m && r1 - k <= w) ? at(r1, k) : 0.0;
            }
            double dg = 0.0;   // D of the lane's own panel column
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const double Dk = readlane_d(a0[b], b);
                dg = t == b ? a0[b] : dg;
                const bool first = t > b;
                const double l = (first ? a0[b] : a1[b]) / Dk;
                const double v = l * Dk;
                const int d = first ? t - b : 64 + t - b;   // the lane's row of the column is k + d
                if (d <= w) {
                    Lp[b][d] = l;
                    vp[b][d] = v;
                }
                const double l1 = first ? 0.0 : l;
                // the terms of column k in the panel's later columns
#pragma unroll
                for (int jb = b + 1; jb < B; ++jb) {
                    const double vj = readlane_d(v, jb);   // v(k0 + jb, k), the lane of row k0 + jb
                    a0[jb] = a0[jb] - l * vj;
                    a1[jb] = a1[jb] - l1 * vj;
                }
            }
            if (t < B) Dpan[t] = dg;
        }
        lds_barrier();
        // the panel's columns go to memory, a row's B entries side by side
        if (t < (w + B - 1) * B) {
            const int r = k0 + 1 + t / B, b = t % B, d = r - k0 - b;
            if (d >= 1 && d <= w && r < m) Lb[(size_t)r * w + (w - d)] = Lp[b][d];
        }
        if (t >= BAND_FACTOR_THREADS - B) {
            const int b = t - (BAND_FACTOR_THREADS - B);
            if (k0 + b < m) {
                const double Dk = Dpan[b];
                D[k0 + b] = Dk;
                if (!(Dk > 0.0)) bad = 1;
            }
        }
        // the panel's terms in the trailing triangle (rows and columns
        // k0 + B .. k0 + B - 1 + w), in column order
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2) {
            const int i = k0 + B - 1 + di[s2], j = k0 + B - 1 + dj[s2];
            if (di[s2] > 0 && i < m) {
                double a = at(i, j);
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int k = k0 + b;
                    if (i - k <= w && k < m) a = a - Lp[b][i - k] * vp[b][j - k];
                }
                at(i, j) = a;
            }
        }
        // the rows of panel p + 1 enter (their slots are those of panel p's
        // rows); the staging buffer of panel p + 2 is filled from the
        // registers and panel p + 3's entries are requested
        if (enters) {
            const int i = (p + 1) * B + w + eb;
            if (i < m) at(i, i - w + eoff) = eu >= 0 ? stage[(p + 1) & 1][eu] : 0.0;
        }
        if (loader) {
            stage[p & 1][t] = pf;
            pf = entering(p + 3, t);
        }
        lds_barrier();
    }
    if (bad) atomicOr(flags, F_BREAK_COARSE);
}

// The factor as the one-wave solve reads it.  Unknowns are padded to M, a
// multiple of 64; lane l keeps the pending values of unknowns 64q + l (block
// q, "current") and 64(q+1) + l (block q+1, "next"), since w <= 64 means an
// unknown only couples to its own block and the neighbouring one.  A step
// subtracts multiples of one final unknown from at most w <= 64 pending ones,
// one per lane, so every step has one row of 64 doubles (CF for the forward
// substitution, CG for the backward one):
//   forward step j = 64q + r:  CF[j][l] = L(64q + l, j)       for l > r (current block),
//                                         L(64q + 64 + l, j)  for l <= r (next block);
//   backward step k = 64q + r: CG[k][l] = L(k, 64q + l)       for l < r (current block),
//                                         L(k, 64q - 64 + l)  for l >= r (previous block);
// zero wherever the entry lies outside the band or the matrix; Dp = D padded
// with ones.  The 64 rows of a block are contiguous (32 KB).
struct BandSolve {
    const double *CF, *CG, *Dp;
    int m, M, nc;
};

__host__ __device__ inline int band_padded(int m) { return (m + 63) & ~63; }

static __global__ void k_band_expand(int nc, const double *__restrict__ Lb, const double *__restrict__ D,
                                     double *__restrict__ CF, double *__restrict__ CG, double *__restrict__ Dp)
{
    const int m = nc * nc, w = nc + 1, M = band_padded(m);
    const int l = threadIdx.x & 63;
    const int s = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);   // step
    if (s >= M) return;
    const int q = s >> 6, r = s & 63;
    // L(i, k) for i - w <= k < i < m, else 0
    auto Lik = [&](int i, int k) -> double {
        return (i < m && k >= 0 && k < i && i - k <= w) ? Lb[(size_t)i * w + (k - i + w)] : 0.0;
    };
    const size_t o = (size_t)s * 64 + l;
    CF[o] = l > r ? Lik(64 * q + l, s) : Lik(64 * q + 64 + l, s);
    CG[o] = l < r ? Lik(s, 64 * q + l) : (q >= 1 ? Lik(s, 64 * q - 64 + l) : 0.0);
    if (l == 0) Dp[s] = s < m ? D[s] : 1.0;
}

// One step: the final value y of lane r is broadcast and y L is removed from
// the pending values, each update one fused multiply-add (p - L y rounded
// once); f0 applies to a0 (current block), f1 to a1.  A lane whose entry is
// zero keeps its value (up to the sign of a zero).
__device__ __forceinline__ void band_step(double &a0, double &a1, double f0, double f1, int r)
{
    const double y = readlane_d(a0, r);
    a0 = fma(-f0, y, a0);
    a1 = fma(-f1, y, a1);
}

// The coarsest solve x = L^-T D^-1 L^-1 b, in the order of the oracle's
// column form: y_i takes its terms over increasing j, z_i = y_i / D_i, x_i
// takes its terms over decreasing k.  Run by one wave (lanes l = 0..63),
// reading the step rows from global memory (the persistent small-level
// kernel, whose coarsest level is small).  Steps of padding unknowns (index
// >= m) change nothing and are skipped.  get(k): right-hand side of unknown
// k < m as FP64; put(k, x): the result; z: M doubles of scratch.
template <typename Get, typename Put>
__device__ void band_solve_direct(const BandSolve &B, Get get, Put put, double *z)
{
    const int l = threadIdx.x & 63, m = B.m, nb = B.M >> 6;
    double a0 = l < m ? get(l) : 0.0;
    double a1 = 64 + l < m ? get(64 + l) : 0.0;
    constexpr int G = 16;   // steps whose rows are requested together
    for (int q = 0; q < nb; ++q) {
        const double *rows = B.CF + (size_t)q * 4096;
        const int nr = min(64, m - 64 * q);
        for (int r0 = 0; r0 < nr; r0 += G) {
            double f[G];
#pragma unroll
            for (int i = 0; i < G; ++i) f[i] = r0 + i < nr ? rows[(r0 + i) * 64 + l] : 0.0;
#pragma unroll
            for (int i = 0; i < G; ++i) {
                const int r = r0 + i;
                if (r < nr) band_step(a0, a1, l > r ? f[i] : 0.0, l > r ? 0.0 : f[i], r);
            }
        }
        z[64 * q + l] = a0 / B.Dp[64 * q + l];
        a0 = a1;
        a1 = 64 * (q + 2) + l < m ? get(64 * (q + 2) + l) : 0.0;
    }
    a0 = z[64 * (nb - 1) + l];
    a1 = nb >= 2 ? z[64 * (nb - 2) + l] : 0.0;
    for (int q = nb - 1; q >= 0; --q) {
        const double *rows = B.CG + (size_t)q * 4096;
        for (int r0 = min(63, m - 1 - 64 * q); r0 >= 0; r0 -= G) {
            double g[G];
#pragma unroll
            for (int i = 0; i < G; ++i) g[i] = r0 - i >= 0 ? rows[(r0 - i) * 64 + l] : 0.0;
#pragma unroll
            for (int i = 0; i < G; ++i) {
                const int r = r0 - i;
                if (r >= 0) band_step(a0, a1, l < r ? g[i] : 0.0, l < r ? 0.0 : g[i], r);
            }
        }
        if (64 * q + l < m) put(64 * q + l, a0);
        a0 = a1;
        a1 = q >= 2 ? z[64 * q - 128 + l] : 0.0;
    }
}

// The coarsest solve as a kernel of its own (the coarsest level is larger
// than the persistent small-level kernel handles, or the basic path runs).
// Wave 0 runs the chain of steps, BAND_CH per phase, reading each step's
// pair of rows (current block, neighbouring block) from LDS, so a step is a
// broadcast and two fused multiply-adds.  The loader waves expand the
// compressed rows of phase c + 1 into the other of two LDS slots meanwhile,
// the global loads of the phases after it already in flight in their
// registers (BAND_INFLIGHT sets), so memory latency stays behind the chain.
// The right-hand side and the pivots are staged in LDS first (z, dpl), so
// the chain itself waits on no global load.  Phases run forward through the blocks (two per block), then backward:
// nch = 4 M / 64 phases, band_phases(nch) barriers on every wave.  Workgroup
// k solves right-hand side k (its arrays ks elements, its stop flag kstop
// ints after the first's).
constexpr int BAND_LOADERS = 8;
constexpr int BAND_SOLVE_THREADS = 64 * (1 + BAND_LOADERS);
constexpr int BAND_CH = 32;
constexpr int BAND_INFLIGHT = 4;
constexpr int BAND_PER_LANE = BAND_CH * 64 / 2 / (64 * BAND_LOADERS);   // double pairs per loader lane per phase

// Barriers of k_coarse_solve on every wave: one before the first phase and
// one after each, rounded up to whole rounds of the loaders' register sets.
__host__ __device__ inline int band_phases(int nch) { return (nch + BAND_INFLIGHT) / BAND_INFLIGHT * BAND_INFLIGHT; }

__host__ __device__ inline size_t band_solve_lds(int M) { return (2 * (size_t)M + 2 * BAND_CH * 128) * sizeof(double); }

// Steps R0 + BAND_CH - 1 .. R0 (DIR < 0) or R0 .. R0 + BAND_CH - 1 of a block;
// row t of the slot holds step R0 + t (current block at [0, 64), the
// neighbouring one at [64, 128)).  Each step's pair of rows is read
// BAND_AHEAD steps before it runs, and the steps keep their order (a
// scheduling barrier after each), so the chain waits on no LDS read: left
// to itself the scheduler reads a row just before its step to save
// registers, and the read's latency joins the chain.  (Forming two steps'
// broadcasts at once, the second from the first by one fused multiply-add
// on the broadcast values, was measured slower: 21 ns per step against 19.6,
// the extra operations costing more issue time than the broadcast saved.)
#ifndef BMG_BAND_AHEAD
#define BMG_BAND_AHEAD 8
#endif
constexpr int BAND_AHEAD = BMG_BAND_AHEAD;
template <int R0, int DIR>
__device__ __forceinline__ void band_phase(double &a0, double &a1, const double *rows, int l)
{
    double f0[BAND_CH], f1[BAND_CH];
    auto row = [&](int i) {
        const int t = DIR > 0 ? i : BAND_CH - 1 - i;
        f0[i] = rows[t * 128 + l];
        f1[i] = rows[t * 128 + 64 + l];
    };
#pragma unroll
    for (int i = 0; i < BAND_AHEAD; ++i) row(i);
#pragma unroll
    for (int i = 0; i < BAND_CH; ++i) {
        if (i + BAND_AHEAD < BAND_CH) row(i + BAND_AHEAD);
        band_step(a0, a1, f0[i], f1[i], R0 + (DIR > 0 ? i : BAND_CH - 1 - i));
        __builtin_amdgcn_sched_barrier(0);
    }
    // both values complete here: the updates of a1 (off the chain) are not
    // deferred past the barrier that follows, which would keep the phase's
    // rows and broadcasts live across it
    asm volatile("" : "+v"(a0), "+v"(a1));
}

template <typename T>
static __global__ __launch_bounds__(BAND_SOLVE_THREADS) void k_coarse_solve(Lev<T> Cl, BandSolve B, size_t ks,
                                                                               const int *stop, int kstop)
{
    const int rk = blockIdx.x;
    if (stopped(stop ? stop + rk * kstop : stop)) return;
    extern __shared__ double band_sm[];
    double *z = band_sm, *dpl = band_sm + B.M, *slot = band_sm + 2 * B.M;
    const int nb = B.M >> 6, nch = 4 * nb;
    const int l = threadIdx.x & 63;
    const int nc = B.nc, m = B.m;
    auto pos = [&](int k) { return (size_t)(k / nc + 1) * Cl.ld + (k % nc + 1); };
    // every wave: the right-hand side as FP64 (zero past m) into z, the padded
    // pivots into dpl, so that the chain reads no global memory
    {
        const T *bv = Cl.b + (size_t)rk * ks;
        for (int k = threadIdx.x; k < B.M; k += BAND_SOLVE_THREADS) {
            z[k] = k < m ? (double)bv[pos(k)] : 0.0;
            dpl[k] = B.Dp[k];
        }
    }
    if (threadIdx.x >= 64) {
        // loaders.  Phase c: block q, half h (steps 32h .. 32h + 31), forward
        // for c < 2 nb, backward after; its rows are the contiguous rows
        // 64q + 32h .. of CF or CG.
        const int t0 = threadIdx.x - 64;
        typedef double v2d __attribute__((ext_vector_type(2)));
        auto where = [&](int c, int &q, int &h, bool &fwd) {
            fwd = c < 2 * nb;
            const int c2 = fwd ? c : c - 2 * nb;
            q = fwd ? c2 >> 1 : nb - 1 - (c2 >> 1);
            h = fwd ? (c2 & 1) : 1 - (c2 & 1);
        };
        // the loads are unconditional (a phase past the last reads the last)
        // and so are the phases, so that the compiler's wait for a set covers
        // that set's loads only and the other sets stay in flight
        v2d buf[BAND_INFLIGHT][BAND_PER_LANE];
        auto request = [&](v2d(&r)[BAND_PER_LANE], int c) {
            int q, h;
            bool fwd;
            where(min(c, nch - 1), q, h, fwd);
            const v2d *g = reinterpret_cast<const v2d *>((fwd ? B.CF : B.CG) + ((size_t)q * 64 + 32 * h) * 64);
#pragma unroll
            for (int e = 0; e < BAND_PER_LANE; ++e) r[e] = g[t0 + e * 64 * BAND_LOADERS];
        };
        // phase c: the rows of phase c, expanded into pairs (current block,
        // neighbouring block), go into slot c & 1 (a slot no longer read once
        // c >= nch); the set then requests phase c + BAND_INFLIGHT
        auto phase = [&](v2d(&r)[BAND_PER_LANE], int c) {
            int q, h;
            bool fwd;
            where(min(c, nch - 1), q, h, fwd);
            double *dst = slot + (size_t)(c & 1) * BAND_CH * 128;
#pragma unroll
            for (int e = 0; e < BAND_PER_LANE; ++e) {
                const int x = t0 + e * 64 * BAND_LOADERS;   // pair x of the phase's 32 x 32 pairs
                const int t = x >> 5, lp = (x & 31) * 2, rr = 32 * h + t;
                v2d c0, c1;
                const bool k0 = fwd ? lp > rr : lp < rr, k1 = fwd ? lp + 1 > rr : lp + 1 < rr;
                c0.x = k0 ? r[e].x : 0.0;
                c1.x = k0 ? 0.0 : r[e].x;
                c0.y = k1 ? r[e].y : 0.0;
                c1.y = k1 ? 0.0 : r[e].y;
                *reinterpret_cast<v2d *>(dst + t * 128 + lp) = c0;
                *reinterpret_cast<v2d *>(dst + t * 128 + 64 + lp) = c1;
            }
            request(r, c + BAND_INFLIGHT);
            lds_barrier();
        };
#pragma unroll
        for (int u = 0; u < BAND_INFLIGHT; ++u) request(buf[u], u);
        for (int c0 = 0; c0 < band_phases(nch); c0 += BAND_INFLIGHT) {
#pragma unroll
            for (int u = 0; u < BAND_INFLIGHT; ++u) phase(buf[u], c0 + u);
        }
        return;
    }
    // wave 0: forward through the blocks, two phases each, then backward
    T *uv = Cl.u + (size_t)rk * ks;
    lds_barrier();                                  // phase 0, b and the pivots are in LDS
    double a0 = z[l], a1 = nb >= 2 ? z[64 + l] : 0.0, bn = nb >= 3 ? z[128 + l] : 0.0;
    for (int q = 0; q < nb; ++q) {
        band_phase<0, 1>(a0, a1, slot, l);
        lds_barrier();
        band_phase<32, 1>(a0, a1, slot + BAND_CH * 128, l);
        z[64 * q + l] = a0 / dpl[64 * q + l];       // b of block q is no longer needed
        a0 = a1;
        a1 = bn;
        bn = q + 3 < nb ? z[64 * (q + 3) + l] : 0.0;
        lds_barrier();
    }
    a0 = z[64 * (nb - 1) + l];
    a1 = nb >= 2 ? z[64 * (nb - 2) + l] : 0.0;
    bn = nb >= 3 ? z[64 * (nb - 3) + l] : 0.0;
    for (int q = nb - 1; q >= 0; --q) {
        band_phase<32, -1>(a0, a1, slot, l);
        lds_barrier();
        band_phase<0, -1>(a0, a1, slot + BAND_CH * 128, l);
        if (64 * q + l < m) uv[pos(64 * q + l)] = (T)a0;
        a0 = a1;
        a1 = bn;
        bn = q >= 3 ? z[64 * (q - 3) + l] : 0.0;
        lds_barrier();
    }
    for (int c = nch + 1; c < band_phases(nch); ++c) lds_barrier();   // the loaders' last phases
}

// ------------------------------------------------------ basic cycle steps
// One colour of four-colour Gauss-Seidel: colour(i,j) = (i mod 2) + 2 (j mod 2).
// s = b; s -= A_d u_d for d = SW, S, SE, W, E, NW, N, NE; u = s / A_O.
template <typename T, bool NINE>
__device__ __forceinline__ T gs_point(const Lev<T> &L, size_t p)
{
    const size_t ld = L.ld;
    const T *u = L.u;
    T s = L.b[p];
    if (NINE) s -= L.SW[p] * u[p - ld - 1];
    s -= L.S[p] * u[p - ld];
    if (NINE) s -= L.NW[p + 1 - ld] * u[p - ld + 1];
    s -= L.W[p] * u[p - 1];
    s -= L.W[p + 1] * u[p + 1];
    if (NINE) s -= L.NW[p] * u[p + ld - 1];
    s -= L.S[p + ld] * u[p + ld];
    if (NINE) s -= L.SW[p + ld + 1] * u[p + ld + 1];
    return s / L.O[p];
}

template <typename T, bool NINE>
static __global__ void k_gs_colour(Lev<T> L, int colour, const int *stop)
{
    if (stopped(stop)) return;
    const int i = ((colour & 1) ? 1 : 2) + 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int j = ((colour >> 1) ? 1 : 2) + 2 * (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (i > L.n || j > L.n) return;
    const size_t p = (size_t)j * L.ld + i;
    L.u[p] = gs_point<T, NINE>(L, p);
}

// r = b - A u, the centre term last.
template <typename T, bool NINE>
__device__ __forceinline__ T residual_point(const Lev<T> &L, const T *u, size_t p)
{
    const size_t ld = L.ld;
    T s = L.b[p];
    if (NINE) s -= L.SW[p] * u[p - ld - 1];
    s -= L.S[p] * u[p - ld];
    if (NINE) s -= L.NW[p + 1 - ld] * u[p - ld + 1];
    s -= L.W[p] * u[p - 1];
    s -= L.W[p + 1] * u[p + 1];
    if (NINE) s -= L.NW[p] * u[p + ld - 1];
    s -= L.S[p + ld] * u[p + ld];
    if (NINE) s -= L.SW[p + ld + 1] * u[p + ld + 1];
    s -= L.O[p] * u[p];
    return s;
}

template <typename T, bool NINE>
static __global__ void k_residual(Lev<T> L, const int *stop)
{
    if (stopped(stop)) return;
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const size_t p = (size_t)j * L.ld + i;
    L.r[p] = residual_point<T, NINE>(L, L.u, p);
}

// b_c(I,J) = P^T r in the term order of Fig. restrict_kernel; u_c = 0.
template <typename T>
static __global__ void k_restrict(const T *__restrict__ r, int ldf, Wts<T> C, Lev<T> Cl, const int *stop)
{
    if (stopped(stop)) return;
    const int I = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int J = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (I > Cl.n || J > Cl.n) return;
    const size_t c = (size_t)J * C.ld + I;
    const size_t f = (size_t)(2 * J) * ldf + 2 * I;
    const size_t cn = c + C.ld;
    T s = C.at(LNE, c) * r[f - ldf - 1];
    s = s + C.at(LA, c) * r[f - ldf];
    s = s + C.at(LNW, c + 1) * r[f - ldf + 1];
    s = s + C.at(LR, c) * r[f - 1];
    s = s + r[f];
    s = s + C.at(LL, c + 1) * r[f + 1];
    s = s + C.at(LSE, cn) * r[f + ldf - 1];
    s = s + C.at(LB, cn) * r[f + ldf];
    s = s + C.at(LSW, cn + 1) * r[f + ldf + 1];
    Cl.b[c] = s;
    Cl.u[c] = (T)0;
}

// Correction e = P e_c at fine (i,j); e_c is zero on the ring.
template <typename T>
__device__ __forceinline__ T interp_point(const Wts<T> &C, const T *ec, int i, int j)
{
    const int ldc = C.ld;
    if (!(i & 1) && !(j & 1)) return ec[(size_t)(j >> 1) * ldc + (i >> 1)];
    if ((i & 1) && !(j & 1)) {
        const size_t c = (size_t)(j >> 1) * ldc + ((i + 1) >> 1);
        return C.at(LL, c) * ec[c - 1] + C.at(LR, c) * ec[c];
    }
    if (!(i & 1)) {
        const size_t c = (size_t)((j + 1) >> 1) * ldc + (i >> 1);
        return C.at(LB, c) * ec[c - ldc] + C.at(LA, c) * ec[c];
    }
    const size_t c = (size_t)((j + 1) >> 1) * ldc + ((i + 1) >> 1);
    T e = C.at(LSW, c) * ec[c - ldc - 1] + C.at(LSE, c) * ec[c - ldc];
    e = e + C.at(LNW, c) * ec[c - 1];
    e = e + C.at(LNE, c) * ec[c];
    return e;
}

// u += P e_c by coarse cells: thread (I, J) takes the fine points
// (2I-1, 2J-1), (2I, 2J-1), (2I-1, 2J), (2I, 2J), I, J = 1 .. nc+1, whose
// terms all use the weights and e_c around coarse index c = J ldc + I (the
// expressions of interp_point), so a wave runs no divergent paths; fine
// points on the ring (column or row n+1) are skipped.
template <typename T>
static __global__ void k_interp_add(Lev<T> L, Wts<T> C, const T *__restrict__ ec, const int *stop)
{
    if (stopped(stop)) return;
    const int I = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int J = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    const int n = L.n, nc = (n - 1) / 2;
    if (I > nc + 1 || J > nc + 1) return;
    const int ldc = C.ld;
    const size_t c = (size_t)J * ldc + I;
    const T e00 = ec[c], e01 = ec[c - 1], e10 = ec[c - ldc], e11 = ec[c - ldc - 1];
    const size_t p = (size_t)(2 * J - 1) * L.ld + (2 * I - 1);   // the odd-odd point
    const bool east = 2 * I <= n, north = 2 * J <= n;
    {
        T e = C.at(LSW, c) * e11 + C.at(LSE, c) * e10;
        e = e + C.at(LNW, c) * e01;
        e = e + C.at(LNE, c) * e00;
        L.u[p] = L.u[p] + e;
    }
    if (east) L.u[p + 1] = L.u[p + 1] + (C.at(LB, c) * e10 + C.at(LA, c) * e00);
    if (north) L.u[p + L.ld] = L.u[p + L.ld] + (C.at(LL, c) * e01 + C.at(LR, c) * e00);
    if (east && north) L.u[p + L.ld + 1] = L.u[p + L.ld + 1] + e00;
}

// k_interp_add over the coarse cells of fine level F.
template <typename T>
static inline void launch_interp_add(const Lev<T> &F, const Wts<T> &C, const T *ec, const int *stop, hipStream_t st)
{
    const int cells = (F.n - 1) / 2 + 1;
    const dim3 blk(64, 4), grid((cells + 63) / 64, (cells + 3) / 4);
    hipLaunchKernelGGL((k_interp_add<T>), grid, blk, 0, st, F, C, ec, stop);
}

// ------------------------------------------------------------ reductions
// Wave64 + LDS block reduction of a double (up to 16 waves) through 16
// doubles of LDS at `part`; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *part)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (wid == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        v = lane < nw ? part[lane] : 0.0;
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    }
    return v;
}

__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double part[16];
    return block_sum(v, part);
}

// Per-block partial sums of squares of the residual (r_mode = 1: recompute
// b - A u; 0: of the array x itself) over the interior, grid-stride over rows.
template <typename T, bool NINE, bool RES>
static __global__ void k_sumsq_partial(Lev<T> L, const T *__restrict__ x, double *__restrict__ part,
                                const int *stop)
{
    if (stopped(stop)) return;
    double acc = 0.0;
    const int n = L.n;
    for (int j = 1 + blockIdx.x; j <= n; j += gridDim.x) {
        for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x) {
            const size_t p = (size_t)j * L.ld + i;
            const double v = RES ? (double)residual_point<T, NINE>(L, L.u, p) : (double)x[p];
            acc += v * v;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Partial sums of s_p^2 with s_p = |b_p| + sum_d |A_d(p)| |x_(p+d)| (the
// nine entries of the row, centre included): eps * sqrt(sum) / ||b|| bounds
// the relative residual that rounding the exact solution to FP64 can leave,
// the floor below which no FP64 vector's residual reliably goes.  An estimate
// only, summed in plain FP64.
template <bool NINE>
static __global__ void k_floor_partial(Lev<double> L, const double *__restrict__ B, const double *__restrict__ X,
                                       double *__restrict__ part)
{
    double acc = 0.0;
    const int n = L.n;
    const size_t ld = L.ld;
    for (int j = 1 + blockIdx.x; j <= n; j += gridDim.x) {
        for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x) {
            const size_t p = (size_t)j * ld + i;
            double s = fabs(B[p]);
            s += fabs(L.S[p]) * fabs(X[p - ld]) + fabs(L.W[p]) * fabs(X[p - 1]);
            s += fabs(L.O[p]) * fabs(X[p]);
            s += fabs(L.W[p + 1]) * fabs(X[p + 1]) + fabs(L.S[p + ld]) * fabs(X[p + ld]);
            if (NINE) {
                s += fabs(L.SW[p]) * fabs(X[p - ld - 1]) + fabs(L.NW[p + 1 - ld]) * fabs(X[p - ld + 1]);
                s += fabs(L.NW[p]) * fabs(X[p + ld - 1]) + fabs(L.SW[p + ld + 1]) * fabs(X[p + ld + 1]);
            }
            acc += s * s;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Several right-hand sides in one launch (block solves): the launch serves
// those whose mode[] equals `want`; right-hand side z's level-0 u, b are kl
// elements after the first's, its B, XH, XL planes kx after, its partial sums
// kpart doubles, scalars kscal doubles, history khist doubles and (count, stop)
// pair kcnt ints after.
struct RhsFan {
    int nrhs;
    const int *mode;
    int want;
    size_t kl, kx;
    int kpart, kscal, khist, kcnt;
};

// Final sum of the partials (fixed order) -> out[0].  With `hist` given (and
// the solve not stopped), this also records rel = sqrt(sum)/bnorm[0] into hist[*count], advances the count,
// and raises *stop: 1 once rel <= tol, 2 if rel is not finite or exceeds
// 1e3 times the initial relative residual bnorm[1], 3 when maxc entries exist,
// 4 once rel <= refine (refine > 0): the solve switches to refinement.
__device__ __forceinline__ void sumsq_final_body(const double *__restrict__ part, int np, double *__restrict__ out,
                                                 double *hist, int *count, int *stop, const double *bnorm,
                                                 double tol, int maxc, double refine)
{
    double v = 0.0;
    for (int t = threadIdx.x; t < np; t += blockDim.x) v += part[t];
    v = block_sum(v);
    if (threadIdx.x == 0) {
        out[0] = v;
        if (hist) {
            const int k = *count;
            const double rel = sqrt(v) / bnorm[0];
            hist[k] = rel;
            *count = k + 1;
            int s = 0;
            if (rel <= tol) s = 1;
            else if (!isfinite(rel) || rel > 1e3 * bnorm[1]) s = 2;
            else if (k + 1 >= maxc) s = 3;
            else if (refine > 0.0 && rel <= refine) s = 4;
            if (s) *stop = s;
        }
    }
}

static __global__ void k_sumsq_final(const double *__restrict__ part, int np, double *__restrict__ out,
                              double *hist, int *count, int *stop, const double *bnorm,
                              double tol, int maxc, double refine)
{
    if (hist && stopped(stop)) return;   // a finished solve records nothing more
    sumsq_final_body(part, np, out, hist, count, stop, bnorm, tol, maxc, refine);
}

// The same for the right-hand sides F selects (one workgroup each): out and
// bnorm are the first right-hand side's, count its (count, stop) pair.
static __global__ void k_sumsq_final_fan(const double *__restrict__ part, int np, double *out, double *hist,
                                         int *count, const double *bnorm, double tol, int maxc, double refine,
                                         RhsFan F)
{
    const int z = blockIdx.x;
    int *cz = count + z * F.kcnt;
    if (F.mode[z] != F.want || stopped(cz + 1)) return;
    sumsq_final_body(part + (size_t)z * F.kpart, np, out + z * F.kscal, hist + (size_t)z * F.khist, cz, cz + 1,
                     bnorm + z * F.kscal, tol, maxc, refine);
}

// ---------------------------------------------------- layout conversions
// [n][n] user array <-> padded level array.
template <typename TI, typename TO>
static __global__ void k_pack_in(const TI *__restrict__ src, int n, TO *__restrict__ dst, int ld)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > n || j > n) return;
    dst[(size_t)j * ld + i] = (TO)src[(size_t)(j - 1) * n + (i - 1)];
}

template <typename TI, typename TO>
static __global__ void k_pack_out(const TI *__restrict__ src, int ld, int n, TO *__restrict__ dst)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > n || j > n) return;
    dst[(size_t)(j - 1) * n + (i - 1)] = (TO)src[(size_t)j * ld + i];
}

// Rounded copy of a padded array (the FP32 hierarchy from the FP64 set-up).
static __global__ void k_round_f32(const double *__restrict__ src, float *__restrict__ dst, size_t count)
{
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count;
         t += (size_t)gridDim.x * blockDim.x)
        dst[t] = (float)src[t];
}

// Up to ROUND_MAX arrays rounded to FP32 in one launch (a hierarchy's
// planes): blockIdx.y selects the array.
constexpr int ROUND_MAX = 96;
struct RoundList {
    int n;
    const double *src[ROUND_MAX];
    float *dst[ROUND_MAX];
    size_t count[ROUND_MAX];
};

static __global__ void k_round_f32_list(RoundList R)
{
    const int a = blockIdx.y;
    if (a >= R.n) return;
    const double *__restrict__ src = R.src[a];
    float *__restrict__ dst = R.dst[a];
    const size_t count = R.count[a];
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count;
         t += (size_t)gridDim.x * blockDim.x)
        dst[t] = (float)src[t];
}

// -------------------------------------------- FP64 iterative refinement
// Maximum over the block (up to 16 waves); result valid in thread 0.
__device__ __forceinline__ double block_max(double m)
{
    __shared__ double sm[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, sm[w]);
    return m;
}

// Largest of np partial maxima of |r| -> out[0] (a maximum: the same value in
// any order of reduction).
static __global__ void k_absmax_final(const double *__restrict__ part, int np, double *__restrict__ out,
                               const int *stop)
{
    if (stopped(stop)) return;
    double m = 0.0;
    for (int t = threadIdx.x; t < np; t += blockDim.x) m = fmax(m, part[t]);
    m = block_max(m);
    if (threadIdx.x == 0) out[0] = m;
}

// Exponent e of the scale 2^e: the least power of two >= rmax (1 for rmax = 0).
__device__ __forceinline__ int ir_exponent(double rmax)
{
    int e = 0;
    const double fr = frexp(rmax, &e);  // rmax = fr 2^e, fr in [1/2, 1)
    if (fr == 0.5) e -= 1;
    if (fr == 0.0) e = 0;
    return e;
}

// s = the smallest power of two >= ||r||_inf (1 if r = 0); the FP32 right-hand
// side is fl32(r / s) (an exact scaling, then one rounding) and u32 = 0.
static __global__ void k_ir_scale(Lev<double> L, Lev<float> F, const double *__restrict__ rmax,
                           double *__restrict__ scale, const int *stop)
{
    if (stopped(stop)) return;
    const int e = ir_exponent(*rmax);
    const double inv = ldexp(1.0, -e);
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i == 1 && j == 1) scale[0] = ldexp(1.0, e);
    if (i > L.n || j > L.n) return;
    const size_t p = (size_t)j * L.ld + i;
    F.b[p] = (float)(L.r[p] * inv);
    F.u[p] = 0.0f;
}

// ------------------------------------------------ double-FP64 iterate
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    const double x = a + b, z = x - a;
    s = x;
    e = (a - (x - z)) + (b - z);
}

// Accurate residual r = B - A (XH + XL) (XL nullable) on the fine level: the
// plain residual's terms in its order (SW, S, SE, W, E, NW, N, NE, centre),
// each product split into value and exact error by fma, each subtraction by
// TwoSum, the errors summed apart, then the XL products, one final rounding.
// MODE 0: sum of squares only; 1: also r -> rout; 2: also r -> L.b and 0 -> L.u
// (the next refinement cycle starts from zero on the right-hand side r).


// Row block rb of nrb (rows 1 + rb, 1 + rb + nrb, ...): the sum of squares of
// r into part[rb] and, with MODE 1 (the refinement of the FP32 cycle, which
// scales r by its largest magnitude next), max |r| into part[nrb + rb].
template <bool NINE, int MODE>
__device__ __forceinline__ void resid_dd_rows(Lev<double> L, const double *__restrict__ B,
                                              const double *__restrict__ XH, const double *__restrict__ XL,
                                              double *__restrict__ rout, double *__restrict__ part, int rb, int nrb)
{
    const size_t ld = L.ld;
    const int n = L.n;
    double acc = 0.0, mx = 0.0;
    for (int j = 1 + rb; j <= n; j += nrb) {
        for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x) {
            const size_t p = (size_t)j * ld + i;
            double a[9];
            size_t q[9] = {p - ld - 1, p - ld, p - ld + 1, p - 1, p + 1, p + ld - 1, p + ld, p + ld + 1, p};
            a[0] = NINE ? L.SW[p] : 0.0;
            a[1] = L.S[p];
            a[2] = NINE ? L.NW[p + 1 - ld] : 0.0;
            a[3] = L.W[p];
            a[4] = L.W[p + 1];
            a[5] = NINE ? L.NW[p] : 0.0;
            a[6] = L.S[p + ld];
            a[7] = NINE ? L.SW[p + ld + 1] : 0.0;
            a[8] = L.O[p];
            double s = B[p], c = 0.0, ns, se;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                if (!NINE && (t == 0 || t == 2 || t == 5 || t == 7)) continue;
                const double x = XH[q[t]];
                const double pr = a[t] * x;
                const double pe = fma(a[t], x, -pr);
                two_sum(s, -pr, ns, se);
                s = ns;
                c = c + (se - pe);
            }
            if (XL) {
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    if (!NINE && (t == 0 || t == 2 || t == 5 || t == 7)) continue;
                    two_sum(s, -(a[t] * XL[q[t]]), ns, se);
                    s = ns;
                    c = c + se;
                }
            }
            const double r = s + c;
            if (MODE == 1) {
                rout[p] = r;
                mx = fmax(mx, fabs(r));
            }
            if (MODE == 2) {
                L.b[p] = r;
                L.u[p] = 0.0;
            }
            acc += r * r;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[rb] = acc;
    if (MODE == 1) {
        mx = block_max(mx);
        if (threadIdx.x == 0) part[nrb + rb] = mx;
    }
}

template <bool NINE, int MODE>
static __global__ void k_resid_dd(Lev<double> L, const double *__restrict__ B, const double *__restrict__ XH,
                           const double *__restrict__ XL, double *__restrict__ rout,
                           double *__restrict__ part, const int *stop)
{
    if (stopped(stop)) return;
    resid_dd_rows<NINE, MODE>(L, B, XH, XL, rout, part, blockIdx.x, gridDim.x);
}

// The same for the right-hand sides F selects: work item w serves right-hand
// side w % nrhs and row block w / nrhs.  Consecutive workgroups are dealt
// round-robin to the 8 XCDs, so w regroups them (grids that are a multiple of
// 8) to give each XCD a contiguous run: the right-hand sides of a row block run
// side by side on one XCD and share its operator rows through that L2.
template <bool NINE, int MODE>
static __global__ void k_resid_dd_fan(Lev<double> L, const double *__restrict__ B, const double *__restrict__ XH,
                                      const double *__restrict__ XL, double *__restrict__ part, const int *stop,
                                      RhsFan F)
{
    const int g = gridDim.x;
    const int w = (g & 7) ? (int)blockIdx.x : (int)(blockIdx.x & 7) * (g >> 3) + (int)(blockIdx.x >> 3);
    const int z = w % F.nrhs;
    if (F.mode[z] != F.want || stopped(stop + z * F.kcnt)) return;
    L.u += z * F.kl;
    L.b += z * F.kl;
    resid_dd_rows<NINE, MODE>(L, B + z * F.kx, XH + z * F.kx, XL ? XL + z * F.kx : XL, nullptr,
                              part + (size_t)z * F.kpart, w / F.nrhs, g / F.nrhs);
}

// (XH, XL) += d in double-FP64 with d = L.u (FP64 inner cycle) or
// d = scale * (double)U32 (FP32 inner cycle): TwoSum, add the low part,
// renormalise with Dekker's fast TwoSum.
__device__ __forceinline__ void dd_update_point(const Lev<double> &L, double *__restrict__ XH,
                                                double *__restrict__ XL, const float *__restrict__ U32,
                                                const double *__restrict__ scale)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const size_t p = (size_t)j * L.ld + i;
    const double d = U32 ? scale[0] * (double)U32[p] : L.u[p];
    double s, e;
    two_sum(XH[p], d, s, e);
    e = e + XL[p];
    const double hi = s + e;
    XL[p] = e - (hi - s);
    XH[p] = hi;
}

static __global__ void k_dd_update(Lev<double> L, double *__restrict__ XH, double *__restrict__ XL,
                            const float *__restrict__ U32, const double *__restrict__ scale,
                            const int *stop)
{
    if (stopped(stop)) return;
    dd_update_point(L, XH, XL, U32, scale);
}

// FP64 inner cycle, the right-hand sides F selects (blockIdx.z).
static __global__ void k_dd_update_fan(Lev<double> L, double *__restrict__ XH, double *__restrict__ XL,
                                       const int *stop, RhsFan F)
{
    const int z = blockIdx.z;
    if (F.mode[z] != F.want || stopped(stop + z * F.kcnt)) return;
    L.u += z * F.kl;
    dd_update_point(L, XH + z * F.kx, XL + z * F.kx, nullptr, nullptr);
}

}  // namespace bmg
