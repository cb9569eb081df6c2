/*
 * CPU oracle for the black-box multigrid (BoxMG) V-cycle on 2D vertex-centred
 * grids, in plain C, FP64 (plus the FP32 V-cycle used inside FP64 iterative
 * refinement).  It follows the method as the paper states it (Section 2 and
 * Fig. vcycle_flowchart: Gauss-Seidel relaxation, residual, restriction,
 * interpolation, a direct coarsest-level solve, coarse operators built by local
 * stencil operations; restriction as in Fig. restrict_kernel; the nine-point
 * stencil of Fig. stencil_operator) with the readings of the unstated parts
 * listed in the design notes: vertex-centred five-point discretisation,
 * operator-induced (collapsed-stencil) interpolation, Galerkin coarse operators
 * P^T A P, four-colour Gauss-Seidel, and a square-root-free Cholesky (LDL^T)
 * of the band matrix of the coarsest grid (3x3 unless set-up asks for a larger
 * one).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source with the
 * HIP library and is written to be read against the paper: plain loops, no
 * blocking, fusion or reordering.
 *
 * Build: gcc -O3 -ffp-contract=off -fopenmp -fPIC -shared (see build.py).
 * Every sum is evaluated left to right as written; division is IEEE division.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EBREAKDOWN (-2)
#define ORC_ENOCONV (-3)
#define ORC_ENOMEM (-7)
#define ORC_MAXL 24

/* ---------------------------------------------------------------- core ops */
#define REAL double
#define SFX(name) name##_d
#include "bmg_oracle_core.inc"
#undef REAL
#undef SFX
#define REAL float
#define SFX(name) name##_f
#include "bmg_oracle_core.inc"
#undef REAL
#undef SFX

static int valid_n(int n);

/* ------------------------------------------------------- line relaxation
 * The "Line" relaxation of Fig. vcycle_flowchart, read as BoxMG's alternating
 * zebra line Gauss-Seidel (FP64): x-lines (rows) with odd index, then even,
 * then y-lines (columns) with odd index, then even.  Each line's equations are
 * solved exactly for its own unknowns with every other unknown at its current
 * value.  A line is a tridiagonal system:
 *   x-line j: a_i = A_W(i,j), b_i = A_O(i,j), c_i = A_E(i,j), i = 1..n;
 *   y-line i: a_j = A_S(i,j), b_j = A_O(i,j), c_j = A_N(i,j), j = 1..n;
 * right-hand side d = b minus the couplings to the two neighbouring lines,
 * the lower (x-line: SW, S, SE) or left (y-line: SW, W, NW) one first, then
 * the upper (NW, N, NE) or right (SE, E, NE) one, each in increasing
 * position.  With this order an x-line is the y-line of the transposed grid.
 *
 * Each line matrix is factored once per level, T = L U (Thomas): m_1 = b_1,
 * l_k = a_k / m_{k-1}, m_k = b_k - l_k c_{k-1}; stored are l_k and the
 * reciprocal pivots r_k = 1 / m_k.  A solve is y_1 = d_1, y_k = d_k - l_k
 * y_{k-1}, then x_n = y_n r_n, x_k = (y_k - c_k x_{k+1}) r_k.  */

/* Factor of every x-line (dir 0) or y-line (dir 1) of a level into the planes
 * l, r ((n+2)^2, entry of unknown k of the line at its grid point).  Returns
 * ORC_EBREAKDOWN if a pivot is not positive and finite. */
static int line_factor_dir(int n, const double *O, const double *W, const double *S, int dir,
                           double *lf, double *rf)
{
    const size_t ld = (size_t)n + 2;
    /* point k of line t, and the strides to the previous / next point */
    const size_t step = dir == 0 ? 1 : ld;
    int bad = 0;
    for (int t = 1; t <= n; ++t) {
        const size_t p0 = dir == 0 ? (size_t)t * ld + 1 : ld + (size_t)t;
        double m_prev = 0.0;
        for (int k = 1; k <= n; ++k) {
            const size_t p = p0 + (size_t)(k - 1) * step;
            /* a_k: the coupling to the previous point; c_{k-1}: the previous
             * point's coupling to this one (the same entry, symmetric) */
            const double a = dir == 0 ? W[p] : S[p];
            double m;
            if (k == 1) {
                lf[p] = 0.0;
                m = O[p];
            } else {
                const double l = a / m_prev;
                lf[p] = l;
                m = O[p] - l * a;
            }
            if (!(m > 0.0) || !isfinite(m)) bad = 1;
            rf[p] = 1.0 / m;
            m_prev = m;
        }
    }
    return bad ? ORC_EBREAKDOWN : ORC_OK;
}

int orc_line_factor(int n, const double *O, const double *W, const double *S,
                    double *lx, double *rx, double *ly, double *ry)
{
    if (!valid_n(n)) return ORC_EINVAL;
    const int a = line_factor_dir(n, O, W, S, 0, lx, rx);
    const int b = line_factor_dir(n, O, W, S, 1, ly, ry);
    return a != ORC_OK ? a : b;
}

/* Solve line t of direction dir (its right-hand side from the current u) and
 * store it into u. */
static void line_solve(int n, const double *O, const double *W, const double *S,
                       const double *SW, const double *NW, const double *lf,
                       const double *rf, const double *b, double *u, int dir, int t,
                       double *y)
{
    (void)O;
    const size_t ld = (size_t)n + 2;
    const size_t step = dir == 0 ? 1 : ld;
    const size_t p0 = dir == 0 ? (size_t)t * ld + 1 : ld + (size_t)t;
    for (int k = 1; k <= n; ++k) {
        const size_t p = p0 + (size_t)(k - 1) * step;
        double d = b[p];
        if (dir == 0) {
            if (SW) d -= SW[p] * u[p - ld - 1];
            d -= S[p] * u[p - ld];
            if (NW) d -= NW[p + 1 - ld] * u[p - ld + 1];   /* A_SE */
            if (NW) d -= NW[p] * u[p + ld - 1];
            d -= S[p + ld] * u[p + ld];                   /* A_N  */
            if (SW) d -= SW[p + ld + 1] * u[p + ld + 1];  /* A_NE */
        } else {
            if (SW) d -= SW[p] * u[p - ld - 1];
            d -= W[p] * u[p - 1];
            if (NW) d -= NW[p] * u[p + ld - 1];
            if (NW) d -= NW[p + 1 - ld] * u[p - ld + 1];   /* A_SE */
            d -= W[p + 1] * u[p + 1];                     /* A_E  */
            if (SW) d -= SW[p + ld + 1] * u[p + ld + 1];  /* A_NE */
        }
        y[k] = k == 1 ? d : d - lf[p] * y[k - 1];
    }
    double x = 0.0;
    for (int k = n; k >= 1; --k) {
        const size_t p = p0 + (size_t)(k - 1) * step;
        const double c = dir == 0 ? W[p + 1] : S[p + ld];   /* A_E or A_N */
        x = k == n ? y[k] * rf[p] : (y[k] - c * x) * rf[p];
        u[p] = x;
    }
}

/* `sweeps` alternating zebra line relaxations of u. */
static void line_relax_sweeps(int n, const double *O, const double *W, const double *S,
                              const double *SW, const double *NW, const double *lx,
                              const double *rx, const double *ly, const double *ry,
                              const double *b, double *u, int sweeps)
{
    for (int sweep = 0; sweep < sweeps; ++sweep) {
        for (int dir = 0; dir < 2; ++dir) {
            for (int parity = 1; parity >= 0; --parity) {   /* odd lines, then even */
#pragma omp parallel
                {
                    double *y = (double *)malloc(((size_t)n + 1) * sizeof(double));
#pragma omp for schedule(static)
                    for (int t = 2 - parity; t <= n; t += 2)
                        line_solve(n, O, W, S, SW, NW, dir == 0 ? lx : ly, dir == 0 ? rx : ry,
                                   b, u, dir, t, y);
                    free(y);
                }
            }
        }
    }
}

void orc_line_relax(int n, const double *O, const double *W, const double *S, const double *SW,
                    const double *NW, const double *lx, const double *rx, const double *ly,
                    const double *ry, const double *b, double *u, int sweeps)
{
    line_relax_sweeps(n, O, W, S, SW, NW, lx, rx, ly, ry, b, u, sweeps);
}

/* Error-free transformations: Knuth's TwoSum and the fma TwoProduct. */
static inline void two_sum_(double a, double b, double *s, double *e)
{
    const double x = a + b, z = x - a;
    *s = x;
    *e = (a - (x - z)) + (b - z);
}

/* Accurate residual r = b - A (xh + xl) on the fine level, xl nullable: the
 * terms of the plain residual in the same order (SW, S, SE, W, E, NW, N, NE,
 * centre), every product split exactly into value and error (TwoProduct by
 * fma), every subtraction into value and error (TwoSum), the errors summed
 * apart, then the products with xl (whose own rounding is below the result's
 * precision), and one final rounding of value + errors (the compensated dot
 * product of Ogita, Rump and Oishi, 2005).  It is as accurate as a residual
 * computed in twice the working precision. */
static void residual_dd(int n, const double *O, const double *W, const double *S,
                        const double *SW, const double *NW, const double *b,
                        const double *xh, const double *xl, double *r)
{
    const size_t ld = (size_t)n + 2;
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= n; ++j) {
        for (int i = 1; i <= n; ++i) {
            const size_t p = (size_t)j * ld + (size_t)i;
            const size_t q[9] = {p - ld - 1, p - ld, p - ld + 1, p - 1, p + 1,
                                 p + ld - 1, p + ld, p + ld + 1, p};
            double a[9];
            a[0] = SW ? SW[p] : 0.0;
            a[1] = S[p];
            a[2] = NW ? NW[p + 1 - ld] : 0.0;
            a[3] = W[p];
            a[4] = W[p + 1];
            a[5] = NW ? NW[p] : 0.0;
            a[6] = S[p + ld];
            a[7] = SW ? SW[p + ld + 1] : 0.0;
            a[8] = O[p];
            double s = b[p], c = 0.0, ns, se;
            for (int t = 0; t < 9; ++t) {
                const double pr = a[t] * xh[q[t]];
                const double pe = fma(a[t], xh[q[t]], -pr);
                two_sum_(s, -pr, &ns, &se);
                s = ns;
                c = c + (se - pe);
            }
            if (xl) {
                for (int t = 0; t < 9; ++t) {
                    two_sum_(s, -(a[t] * xl[q[t]]), &ns, &se);
                    s = ns;
                    c = c + se;
                }
            }
            r[p] = s + c;
        }
    }
}

/* (xh, xl) + d in double-FP64: TwoSum of the high parts, the low part added to
 * the error, then renormalised (Dekker's fast TwoSum). */
static inline void dd_add(double *xh, double *xl, double d)
{
    double s, e;
    two_sum_(*xh, d, &s, &e);
    e = e + *xl;
    const double hi = s + e;
    *xl = e - (hi - s);
    *xh = hi;
}

static int valid_n(int n) { return n >= 3 && ((n + 1) & n) == 0; }

/* ----------------------------------------------------- a0: discretisation */
/* Vertex-centred finite-volume form of -div(k grad u) = f (Section 2, Eq. 1)
 * with cell-constant k: the coupling across the dual-cell face between two
 * neighbouring vertices is minus the mean of the two cells that share the grid
 * edge, A_O is minus the sum of the four couplings (taken before the couplings
 * to the Dirichlet boundary are removed), and b = h^2 f.  No 1/h^2 scaling.
 * Output: stencil [n][n][5] in the order S, W, O, E, N and rhs [n][n]. */
int orc_discretize(int n, const double *k, const double *f, double *st, double *rhs)
{
    if (!valid_n(n)) return ORC_EINVAL;
    const size_t lk = (size_t)n + 1;
    int m = 0;
    while ((1 << m) < n + 1) ++m;
    const double h2 = ldexp(1.0, -2 * m);
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= n; ++j) {
        for (int i = 1; i <= n; ++i) {
            const double kSW = k[(size_t)(j - 1) * lk + (size_t)(i - 1)];
            const double kSE = k[(size_t)(j - 1) * lk + (size_t)i];
            const double kNW = k[(size_t)j * lk + (size_t)(i - 1)];
            const double kNE = k[(size_t)j * lk + (size_t)i];
            double aW = -0.5 * (kSW + kNW);
            double aE = -0.5 * (kSE + kNE);
            double aS = -0.5 * (kSW + kSE);
            double aN = -0.5 * (kNW + kNE);
            const double aO = -(((aW + aE) + aS) + aN);
            if (i == 1) aW = 0.0;
            if (i == n) aE = 0.0;
            if (j == 1) aS = 0.0;
            if (j == n) aN = 0.0;
            double *q = st + ((size_t)(j - 1) * (size_t)n + (size_t)(i - 1)) * 5;
            q[0] = aS; q[1] = aW; q[2] = aO; q[3] = aE; q[4] = aN;
            rhs[(size_t)(j - 1) * (size_t)n + (size_t)(i - 1)] =
                h2 * f[(size_t)(j - 1) * (size_t)n + (size_t)(i - 1)];
        }
    }
    return ORC_OK;
}

/* -------------------------------------------- a1: interpolation weights */
/* Nine entries of row p of a compact stencil, in the order
 * SW, S, SE, W, O, E, NW, N, NE (absent corners of a 5-point level are 0). */
static void row9(size_t ld, const double *O, const double *W, const double *S,
                 const double *SW, const double *NW, size_t p, double a[9])
{
    a[0] = SW ? SW[p] : 0.0;
    a[1] = S[p];
    a[2] = NW ? NW[p + 1 - ld] : 0.0;
    a[3] = W[p];
    a[4] = O[p];
    a[5] = W[p + 1];
    a[6] = NW ? NW[p] : 0.0;
    a[7] = S[p + ld];
    a[8] = SW ? SW[p + ld + 1] : 0.0;
}

/* Positive off-diagonal entries are moved onto the diagonal before the
 * stencil is collapsed (in the order SW,S,SE,W,E,NW,N,NE): the row sum is kept
 * and the collapsed denominators stay positive when a Galerkin operator is not
 * an M-matrix.  On M-matrix rows nothing changes. */
static void lump9(double a[9])
{
    for (int e = 0; e < 9; ++e) {
        if (e == 4) continue;
        if (a[e] > 0.0) {
            a[4] = a[4] + a[e];
            a[e] = 0.0;
        }
    }
}

/* Operator-induced interpolation (the collapsed-stencil construction of the
 * black-box multigrid literature the paper cites in Section 2), applied to the
 * lumped rows.  For the fine F-points around coarse (I,J) = fine (2I,2J):
 *   x-edge X = (2I-1, 2J):  D = A_O + A_N + A_S,
 *       LL = -(A_W + A_NW + A_SW)/D (weight of coarse (I-1,J)),
 *       LR = -(A_E + A_NE + A_SE)/D (weight of coarse (I,J));
 *   y-edge Y = (2I, 2J-1):  D = A_O + A_W + A_E,
 *       LB = -(A_S + A_SW + A_SE)/D (weight of (I,J-1)),
 *       LA = -(A_N + A_NW + A_NE)/D (weight of (I,J));
 *   cell centre Z = (2I-1, 2J-1), using the edge weights already formed:
 *       LNE = -(A_NE + A_N LR(I,J)   + A_E LA(I,J))   / A_O
 *       LNW = -(A_NW + A_N LL(I,J)   + A_W LA(I-1,J)) / A_O
 *       LSE = -(A_SE + A_S LR(I,J-1) + A_E LB(I,J))   / A_O
 *       LSW = -(A_SW + A_S LL(I,J-1) + A_W LB(I-1,J)) / A_O
 * The weights are stored at the coarse point to the north-east of each F-point
 * triple, the layout the restriction of Fig. restrict_kernel reads
 * (Ci(ic+1,...), Ci(...,jc+1)), for I, J up to nc+1.  Plane order:
 * LNE, LA, LNW, LR, LL, LSE, LB, LSW.  SW/NW null means a 5-point stencil.
 * Returns ORC_EBREAKDOWN if a denominator is not positive. */
int orc_interp_weights(int nf, const double *O, const double *W, const double *S,
                       const double *SW, const double *NW, double *Ci)
{
    if (!valid_n(nf) || nf < 7) return ORC_EINVAL;
    const int nc = (nf - 1) / 2;
    const size_t ldf = (size_t)nf + 2, ldc = (size_t)nc + 2, pl = ldc * ldc;
    double *LNE = Ci, *LA = Ci + pl, *LNW = Ci + 2 * pl, *LR = Ci + 3 * pl;
    double *LL = Ci + 4 * pl, *LSE = Ci + 5 * pl, *LB = Ci + 6 * pl, *LSW = Ci + 7 * pl;
    memset(Ci, 0, 8 * pl * sizeof(double));
    int bad = 0;
    enum { SWd = 0, Sd, SEd, Wd, Od, Ed, NWd, Nd, NEd };
    /* x-edges: I = 1..nc+1, J = 1..nc ; y-edges: I = 1..nc, J = 1..nc+1 */
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int J = 1; J <= nc + 1; ++J) {
        for (int I = 1; I <= nc + 1; ++I) {
            const size_t c = (size_t)J * ldc + (size_t)I;
            double a[9];
            if (J <= nc) {
                const size_t p = (size_t)(2 * J) * ldf + (size_t)(2 * I - 1);
                row9(ldf, O, W, S, SW, NW, p, a);
                lump9(a);
                const double D = (a[Od] + a[Nd]) + a[Sd];
                if (!(D > 0.0)) bad = 1;
                LL[c] = -((a[Wd] + a[NWd]) + a[SWd]) / D;
                LR[c] = -((a[Ed] + a[NEd]) + a[SEd]) / D;
            }
            if (I <= nc) {
                const size_t p = (size_t)(2 * J - 1) * ldf + (size_t)(2 * I);
                row9(ldf, O, W, S, SW, NW, p, a);
                lump9(a);
                const double D = (a[Od] + a[Wd]) + a[Ed];
                if (!(D > 0.0)) bad = 1;
                LB[c] = -((a[Sd] + a[SWd]) + a[SEd]) / D;
                LA[c] = -((a[Nd] + a[NWd]) + a[NEd]) / D;
            }
        }
    }
    /* cell centres: I, J = 1..nc+1 */
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int J = 1; J <= nc + 1; ++J) {
        for (int I = 1; I <= nc + 1; ++I) {
            const size_t c = (size_t)J * ldc + (size_t)I;
            const size_t p = (size_t)(2 * J - 1) * ldf + (size_t)(2 * I - 1);
            double a[9];
            row9(ldf, O, W, S, SW, NW, p, a);
            lump9(a);
            if (!(a[Od] > 0.0)) bad = 1;
            LNE[c] = -((a[NEd] + a[Nd] * LR[c]) + a[Ed] * LA[c]) / a[Od];
            LNW[c] = -((a[NWd] + a[Nd] * LL[c]) + a[Wd] * LA[c - 1]) / a[Od];
            LSE[c] = -((a[SEd] + a[Sd] * LR[c - ldc]) + a[Ed] * LB[c]) / a[Od];
            LSW[c] = -((a[SWd] + a[Sd] * LL[c - ldc]) + a[Wd] * LB[c - 1]) / a[Od];
        }
    }
    return bad ? ORC_EBREAKDOWN : ORC_OK;
}

/* ------------------------------------------------------ a2: Galerkin RAP */
/* Weight P(q; K) of coarse basis function K at fine point q, for q in the 3x3
 * fine patch centred on 2K (unit at the coarse point itself). */
static double pweight(const double *Ci, size_t ldc, int KI, int KJ, int qi, int qj)
{
    const size_t pl = ldc * ldc;
    const int di = qi - 2 * KI, dj = qj - 2 * KJ;
#define CI(plane, I, J) Ci[(size_t)(plane) * pl + (size_t)(J) * ldc + (size_t)(I)]
    if (dj == 0) {
        if (di == 0) return 1.0;
        if (di < 0) return CI(3, KI, KJ);          /* LR at X(K)          */
        return CI(4, KI + 1, KJ);                  /* LL at X(K + x)      */
    }
    if (dj < 0) {
        if (di == 0) return CI(1, KI, KJ);         /* LA at Y(K)          */
        if (di < 0) return CI(0, KI, KJ);          /* LNE at Z(K)         */
        return CI(2, KI + 1, KJ);                  /* LNW at Z(K + x)     */
    }
    if (di == 0) return CI(6, KI, KJ + 1);         /* LB at Y(K + y)      */
    if (di < 0) return CI(5, KI, KJ + 1);          /* LSE at Z(K + y)     */
    return CI(7, KI + 1, KJ + 1);                  /* LSW at Z(K + x + y) */
#undef CI
}

/* Galerkin coarse operator A_c = P^T A P, evaluated per coarse point (I,J) and
 * stored direction d in {O, W, S, SW, NW} (the remaining four follow from
 * symmetry):
 *   A_c(I,J;d) = sum_{p in patch(I,J)} P(p;IJ) * sum_{q ~ p, q in supp(K)} A(p,q) P(q;K)
 * with K = (I,J)+d, p over the 3x3 fine patch around (2I,2J) with j outer and i
 * inner, q over p's nine neighbours in the order SW,S,SE,W,O,E,NW,N,NE, both
 * sums starting from zero.  Couplings to ring coarse points are dropped (set
 * to zero), as the Dirichlet boundary requires.  Output is a 9-point level. */
int orc_rap(int nf, const double *O, const double *W, const double *S,
            const double *SW, const double *NW, const double *Ci,
            double *cO, double *cW, double *cS, double *cSW, double *cNW)
{
    if (!valid_n(nf) || nf < 7) return ORC_EINVAL;
    const int nc = (nf - 1) / 2;
    const size_t ldf = (size_t)nf + 2, ldc = (size_t)nc + 2, plc = ldc * ldc;
    memset(cO, 0, plc * sizeof(double));
    memset(cW, 0, plc * sizeof(double));
    memset(cS, 0, plc * sizeof(double));
    memset(cSW, 0, plc * sizeof(double));
    memset(cNW, 0, plc * sizeof(double));
    static const int offI[5] = {0, -1, 0, -1, -1};
    static const int offJ[5] = {0, 0, -1, -1, 1};
#pragma omp parallel for schedule(static)
    for (int J = 1; J <= nc; ++J) {
        for (int I = 1; I <= nc; ++I) {
            double *outs[5] = {cO, cW, cS, cSW, cNW};
            for (int d = 0; d < 5; ++d) {
                const int KI = I + offI[d], KJ = J + offJ[d];
                double acc = 0.0;
                if (KI >= 1 && KJ >= 1 && KJ <= nc) {
                    for (int jj = -1; jj <= 1; ++jj) {
                        for (int ii = -1; ii <= 1; ++ii) {
                            const int pi = 2 * I + ii, pj = 2 * J + jj;
                            const size_t p = (size_t)pj * ldf + (size_t)pi;
                            const double wp = pweight(Ci, ldc, I, J, pi, pj);
                            /* the nine stencil entries of row p, SW..NE */
                            double a[9];
                            row9(ldf, O, W, S, SW, NW, p, a);
                            double t = 0.0;
                            for (int e = 0; e < 9; ++e) {
                                const int qi = pi + (e % 3) - 1, qj = pj + (e / 3) - 1;
                                if (abs(qi - 2 * KI) > 1 || abs(qj - 2 * KJ) > 1) continue;
                                t = t + a[e] * pweight(Ci, ldc, KI, KJ, qi, qj);
                            }
                            acc = acc + wp * t;
                        }
                    }
                }
                outs[d][(size_t)J * ldc + (size_t)I] = acc;
            }
        }
    }
    return ORC_OK;
}

/* ----------------------------------------- a3/a7: coarsest direct solve */
/* The coarsest level is solved directly (Fig. vcycle_flowchart: a Cholesky
 * factorisation; Section 2: a direct solve on a small system).  Its n_L x n_L
 * interior unknowns are numbered lexicographically, k = (i-1) + n_L (j-1), so
 * the nine-point matrix is a band matrix of half-bandwidth w = n_L + 1 and
 * its Cholesky factor has no entries outside that band.
 *
 * Band storage of the lower triangle: row i keeps A_ik for k = i-w .. i at
 * Ab[i (w+1) + (k - i + w)] (diagonal last), entries with k < 0 zero.  The
 * factor keeps L_ik for k = i-w .. i-1 at Lb[i w + (k - i + w)] (the unit
 * diagonal is implicit) and D_i at D[i]. */
static void coarse_band_matrix(int nc, const double *O, const double *W, const double *S,
                               const double *SW, const double *NW, double *Ab)
{
    const size_t ld = (size_t)nc + 2;
    const int w = nc + 1, m = nc * nc;
    memset(Ab, 0, (size_t)m * (size_t)(w + 1) * sizeof(double));
    for (int j = 1; j <= nc; ++j) {
        for (int i = 1; i <= nc; ++i) {
            const size_t p = (size_t)j * ld + (size_t)i;
            const int k = (i - 1) + nc * (j - 1);
            /* the row's couplings to unknowns numbered before it, and A_kk:
             * SW, S, SE (the NW entry of the point below-right), W, O */
            const double ent[5] = {SW ? SW[p] : 0.0, S[p], NW ? NW[p + 1 - ld] : 0.0, W[p], O[p]};
            const int di[5] = {-1, 0, 1, -1, 0}, dj[5] = {-1, -1, -1, 0, 0};
            for (int e = 0; e < 5; ++e) {
                const int qi = i + di[e], qj = j + dj[e];
                if (qi < 1 || qi > nc || qj < 1 || qj > nc) continue;
                const int q = (qi - 1) + nc * (qj - 1);
                Ab[(size_t)k * (w + 1) + (size_t)(q - k + w)] = ent[e];
            }
        }
    }
}

/* Square-root-free Cholesky A = L D L^T of an SPD band matrix (m unknowns,
 * half-bandwidth w), column by column (the form needs only +, -, *, /, so it
 * rounds identically everywhere):
 *   v_k  = L_jk D_k                                   (k = j-w .. j-1)
 *   D_j  = A_jj - sum_k L_jk v_k                      (k increasing)
 *   L_ij = (A_ij - sum_k L_ik v_k) / D_j,  i = j+1 .. j+w, k = i-w .. j-1 increasing.
 * Returns ORC_EBREAKDOWN if a pivot is not positive. */
int orc_band_ldlt_factor(int m, int w, const double *Ab, double *Lb, double *D)
{
    if (m < 1 || w < 1) return ORC_EINVAL;
    double *v = (double *)malloc((size_t)m * sizeof(double));
    if (!v) return ORC_ENOMEM;
    memset(Lb, 0, (size_t)m * (size_t)w * sizeof(double));
#define AB(i, k) Ab[(size_t)(i) * (w + 1) + (size_t)((k) - (i) + w)]
#define LB(i, k) Lb[(size_t)(i) * w + (size_t)((k) - (i) + w)]
    int st = ORC_OK;
    for (int j = 0; j < m && st == ORC_OK; ++j) {
        const int k0 = j - w > 0 ? j - w : 0;
        for (int k = k0; k < j; ++k) v[k] = LB(j, k) * D[k];
        double s = AB(j, j);
        for (int k = k0; k < j; ++k) s = s - LB(j, k) * v[k];
        if (!(s > 0.0)) st = ORC_EBREAKDOWN;
        D[j] = s;
        const int i1 = j + w < m - 1 ? j + w : m - 1;
        for (int i = j + 1; i <= i1; ++i) {
            double t = AB(i, j);
            for (int k = i - w > 0 ? i - w : 0; k < j; ++k) t = t - LB(i, k) * v[k];
            LB(i, j) = t / s;
        }
    }
    free(v);
    return st;
}

/* Solve with the band factor, both triangles in column (axpy) form: once an
 * unknown is final, its multiples are removed from the pending right-hand
 * sides of the unknowns it couples to.
 *   forward:  y = b; for j = 0 .. m-1: y_i -= L_ij y_j   (i = j+1 .. j+w)
 *   scaling:  z_i = y_i / D_i
 *   backward: x = z; for k = m-1 .. 0: x_i -= L_ki x_k   (i = k-w .. k-1)
 * so y_i sums its terms with j increasing and x_i with k decreasing.  Each
 * update is one fused multiply-add, y_i - L_ij y_j rounded once (C99 fma, the
 * correctly rounded operation of IEEE 754-2008). */
void orc_band_ldlt_solve(int m, int w, const double *Lb, const double *D, const double *b, double *x)
{
    for (int i = 0; i < m; ++i) x[i] = b[i];
    for (int j = 0; j < m; ++j) {
        const int i1 = j + w < m - 1 ? j + w : m - 1;
        for (int i = j + 1; i <= i1; ++i) x[i] = fma(-LB(i, j), x[j], x[i]);
    }
    for (int i = 0; i < m; ++i) x[i] = x[i] / D[i];
    for (int k = m - 1; k >= 0; --k) {
        for (int i = k - w > 0 ? k - w : 0; i < k; ++i) x[i] = fma(-LB(k, i), x[k], x[i]);
    }
#undef AB
#undef LB
}

/* ------------------------------------------------------------ a9: norms */
/* Error-free transformations (Knuth TwoSum, TwoProduct by fma) for an
 * accurately rounded sum of squares: the sum is carried as a value plus a
 * running compensation per row, and the rows are combined in row order, so
 * the result does not depend on the thread count. */
static inline void two_sum(double a, double b, double *s, double *e)
{
    const double x = a + b, z = x - a;
    *s = x;
    *e = (a - (x - z)) + (b - z);
}

double orc_sumsq(int n, const double *r)
{
    const size_t ld = (size_t)n + 2;
    double *rs = (double *)malloc((size_t)n * 2 * sizeof(double));
    if (!rs) return NAN;
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= n; ++j) {
        double s = 0.0, c = 0.0;
        for (int i = 1; i <= n; ++i) {
            const double v = r[(size_t)j * ld + (size_t)i];
            const double pr = v * v, pe = fma(v, v, -pr);
            double t, e;
            two_sum(s, pr, &t, &e);
            s = t;
            c = c + (e + pe);
        }
        rs[2 * (j - 1)] = s;
        rs[2 * (j - 1) + 1] = c;
    }
    double s = 0.0, c = 0.0;
    for (int j = 0; j < n; ++j) {
        double t, e;
        two_sum(s, rs[2 * j], &t, &e);
        s = t;
        c = c + (e + rs[2 * j + 1]);
    }
    free(rs);
    return s + c;
}

/* --------------------------------------------------- exported core ops */
void orc_gs(int n, const double *O, const double *W, const double *S,
            const double *SW, const double *NW, const double *b, double *u, int sweeps)
{ gs_sweeps_d(n, O, W, S, SW, NW, b, u, sweeps); }
void orc_residual(int n, const double *O, const double *W, const double *S,
                  const double *SW, const double *NW, const double *b,
                  const double *u, double *r)
{ residual_d(n, O, W, S, SW, NW, b, u, r); }
void orc_restrict(int nf, const double *Ci, const double *r, double *bc)
{ restrict__d(nf, Ci, r, bc); }
void orc_interp_add(int nf, const double *Ci, const double *ec, double *u)
{ interp_add_d(nf, Ci, ec, u); }
void orc_gs_f(int n, const float *O, const float *W, const float *S,
              const float *SW, const float *NW, const float *b, float *u, int sweeps)
{ gs_sweeps_f(n, O, W, S, SW, NW, b, u, sweeps); }
void orc_residual_f(int n, const float *O, const float *W, const float *S,
                    const float *SW, const float *NW, const float *b,
                    const float *u, float *r)
{ residual_f(n, O, W, S, SW, NW, b, u, r); }
void orc_restrict_f(int nf, const float *Ci, const float *r, float *bc)
{ restrict__f(nf, Ci, r, bc); }
void orc_interp_add_f(int nf, const float *Ci, const float *ec, float *u)
{ interp_add_f(nf, Ci, ec, u); }

/* ------------------------------------------------------------ hierarchy */
typedef struct {
    int nlev;
    int n[ORC_MAXL];
    double *O[ORC_MAXL], *W[ORC_MAXL], *S[ORC_MAXL], *SW[ORC_MAXL], *NW[ORC_MAXL];
    double *Ci[ORC_MAXL];             /* weights between level l and l+1 */
    double *u[ORC_MAXL], *b[ORC_MAXL], *r[ORC_MAXL];
    /* FP32 copy of the hierarchy, the FP64 setup rounded to nearest */
    float *fO[ORC_MAXL], *fW[ORC_MAXL], *fS[ORC_MAXL], *fSW[ORC_MAXL], *fNW[ORC_MAXL];
    float *fCi[ORC_MAXL], *fu[ORC_MAXL], *fb[ORC_MAXL], *fr[ORC_MAXL];
    int have_f32;
    /* band LDL^T factor of the coarsest level: m = n_L^2 unknowns,
     * half-bandwidth w = n_L + 1 */
    double *Lb, *Db;
    int cm, cw;
    int nu1, nu2;
    /* line relaxation instead of point Gauss-Seidel: factors of every line */
    int line;
    double *lx[ORC_MAXL], *rx[ORC_MAXL], *ly[ORC_MAXL], *ry[ORC_MAXL];
} orc_hier;

static double *zalloc(size_t count)
{
    return (double *)calloc(count ? count : 1, sizeof(double));
}

void orc_destroy(orc_hier *H)
{
    if (!H) return;
    for (int l = 0; l < ORC_MAXL; ++l) {
        free(H->O[l]); free(H->W[l]); free(H->S[l]); free(H->SW[l]); free(H->NW[l]);
        free(H->Ci[l]); free(H->u[l]); free(H->b[l]); free(H->r[l]);
        free(H->fO[l]); free(H->fW[l]); free(H->fS[l]); free(H->fSW[l]); free(H->fNW[l]);
        free(H->fCi[l]); free(H->fu[l]); free(H->fb[l]); free(H->fr[l]);
        free(H->lx[l]); free(H->rx[l]); free(H->ly[l]); free(H->ry[l]);
    }
    free(H->Lb);
    free(H->Db);
    free(H);
}

int orc_num_levels(const orc_hier *H) { return H->nlev; }
int orc_level_n(const orc_hier *H, int l) { return (l >= 0 && l < H->nlev) ? H->n[l] : -1; }

/* Pointers to the arrays of a level: field 0..4 = O, W, S, SW, NW;
 * 5 = Ci (weights toward level l+1); 6 = u; 7 = b; 8 = r. */
double *orc_field(orc_hier *H, int l, int field)
{
    if (l < 0 || l >= H->nlev) return NULL;
    switch (field) {
    case 0: return H->O[l];
    case 1: return H->W[l];
    case 2: return H->S[l];
    case 3: return H->SW[l];
    case 4: return H->NW[l];
    case 5: return H->Ci[l];
    case 6: return H->u[l];
    case 7: return H->b[l];
    case 8: return H->r[l];
    default: return NULL;
    }
}

/* The coarsest factor: m w entries of L (band storage, see above), then m of
 * D.  *m and *w (nullable) receive the sizes. */
void orc_coarse_factor(const orc_hier *H, double *Lb, double *D, int *m, int *w)
{
    if (Lb) memcpy(Lb, H->Lb, (size_t)H->cm * (size_t)H->cw * sizeof(double));
    if (D) memcpy(D, H->Db, (size_t)H->cm * sizeof(double));
    if (m) *m = H->cm;
    if (w) *w = H->cw;
}

/* Setup: copy the fine operator from the [n][n][K] stencil (K=5: S,W,O,E,N;
 * K=9: SW,S,SE,W,O,E,NW,N,NE) into compact form, then per level form the
 * interpolation weights and the Galerkin coarse operator, down to the
 * coarsest level of nc points per side (nc = 2^k - 1, 3 <= nc <= n), and
 * factor the coarsest matrix.  *status receives the first failure. */
orc_hier *orc_setup(int n, int K, const double *st, int nu1, int nu2, int nc, int *status)
{
    *status = ORC_EINVAL;
    if (!valid_n(n) || (K != 5 && K != 9) || !valid_n(nc) || nc > n) return NULL;
    orc_hier *H = (orc_hier *)calloc(1, sizeof(orc_hier));
    if (!H) { *status = ORC_ENOMEM; return NULL; }
    H->nu1 = nu1; H->nu2 = nu2;
    int nl = 0;
    for (int m = n; m >= nc; m = (m - 1) / 2) H->n[nl++] = m;
    H->nlev = nl;
    for (int l = 0; l < nl; ++l) {
        const size_t sz = (size_t)(H->n[l] + 2) * (size_t)(H->n[l] + 2);
        H->O[l] = zalloc(sz); H->W[l] = zalloc(sz); H->S[l] = zalloc(sz);
        if (l > 0 || K == 9) { H->SW[l] = zalloc(sz); H->NW[l] = zalloc(sz); }
        H->u[l] = zalloc(sz); H->b[l] = zalloc(sz); H->r[l] = zalloc(sz);
        if (l + 1 < nl) {
            const size_t szc = (size_t)(H->n[l + 1] + 2) * (size_t)(H->n[l + 1] + 2);
            H->Ci[l] = zalloc(8 * szc);
        }
    }
    const size_t ld = (size_t)n + 2;
    for (int j = 1; j <= n; ++j) {
        for (int i = 1; i <= n; ++i) {
            const double *q = st + ((size_t)(j - 1) * n + (size_t)(i - 1)) * (size_t)K;
            const size_t p = (size_t)j * ld + (size_t)i;
            if (K == 5) {
                H->S[0][p] = q[0]; H->W[0][p] = q[1]; H->O[0][p] = q[2];
            } else {
                H->SW[0][p] = q[0]; H->S[0][p] = q[1]; H->W[0][p] = q[3];
                H->O[0][p] = q[4]; H->NW[0][p] = q[6];
            }
        }
    }
    for (int l = 0; l + 1 < nl; ++l) {
        int st_w = orc_interp_weights(H->n[l], H->O[l], H->W[l], H->S[l], H->SW[l],
                                      H->NW[l], H->Ci[l]);
        if (st_w != ORC_OK) { *status = st_w; orc_destroy(H); return NULL; }
        orc_rap(H->n[l], H->O[l], H->W[l], H->S[l], H->SW[l], H->NW[l], H->Ci[l],
                H->O[l + 1], H->W[l + 1], H->S[l + 1], H->SW[l + 1], H->NW[l + 1]);
    }
    const int L = nl - 1;
    H->cm = nc * nc;
    H->cw = nc + 1;
    double *Ab = (double *)calloc((size_t)H->cm * (size_t)(H->cw + 1), sizeof(double));
    H->Lb = zalloc((size_t)H->cm * (size_t)H->cw);
    H->Db = zalloc((size_t)H->cm);
    if (!Ab || !H->Lb || !H->Db) { free(Ab); *status = ORC_ENOMEM; orc_destroy(H); return NULL; }
    coarse_band_matrix(nc, H->O[L], H->W[L], H->S[L], H->SW[L], H->NW[L], Ab);
    int st_c = orc_band_ldlt_factor(H->cm, H->cw, Ab, H->Lb, H->Db);
    free(Ab);
    if (st_c != ORC_OK) { *status = st_c; orc_destroy(H); return NULL; }
    *status = ORC_OK;
    return H;
}

/* Relax with alternating zebra line Gauss-Seidel on every level (the FP64
 * cycle): factor every line of every level. */
int orc_set_line_relax(orc_hier *H)
{
    for (int l = 0; l < H->nlev; ++l) {
        const size_t sz = (size_t)(H->n[l] + 2) * (size_t)(H->n[l] + 2);
        if (!H->lx[l]) {
            H->lx[l] = zalloc(sz); H->rx[l] = zalloc(sz); H->ly[l] = zalloc(sz); H->ry[l] = zalloc(sz);
        }
        const int st = orc_line_factor(H->n[l], H->O[l], H->W[l], H->S[l], H->lx[l], H->rx[l],
                                       H->ly[l], H->ry[l]);
        if (st != ORC_OK) return st;
    }
    H->line = 1;
    return ORC_OK;
}

/* The relaxation of level l: point or line Gauss-Seidel. */
static void relax_d(orc_hier *H, int l, int sweeps)
{
    const int n = H->n[l];
    if (H->line)
        line_relax_sweeps(n, H->O[l], H->W[l], H->S[l], H->SW[l], H->NW[l], H->lx[l], H->rx[l],
                          H->ly[l], H->ry[l], H->b[l], H->u[l], sweeps);
    else
        gs_sweeps_d(n, H->O[l], H->W[l], H->S[l], H->SW[l], H->NW[l], H->b[l], H->u[l], sweeps);
}

/* Round the FP64 hierarchy to an FP32 copy (round to nearest even). */
int orc_make_f32(orc_hier *H)
{
    if (H->have_f32) return ORC_OK;
    for (int l = 0; l < H->nlev; ++l) {
        const size_t sz = (size_t)(H->n[l] + 2) * (size_t)(H->n[l] + 2);
        float **dst[5] = {&H->fO[l], &H->fW[l], &H->fS[l], &H->fSW[l], &H->fNW[l]};
        double *src[5] = {H->O[l], H->W[l], H->S[l], H->SW[l], H->NW[l]};
        for (int f = 0; f < 5; ++f) {
            if (!src[f]) continue;
            *dst[f] = (float *)calloc(sz, sizeof(float));
            for (size_t t = 0; t < sz; ++t) (*dst[f])[t] = (float)src[f][t];
        }
        H->fu[l] = (float *)calloc(sz, sizeof(float));
        H->fb[l] = (float *)calloc(sz, sizeof(float));
        H->fr[l] = (float *)calloc(sz, sizeof(float));
        if (H->Ci[l]) {
            const size_t szc = 8 * (size_t)(H->n[l + 1] + 2) * (size_t)(H->n[l + 1] + 2);
            H->fCi[l] = (float *)calloc(szc, sizeof(float));
            for (size_t t = 0; t < szc; ++t) H->fCi[l][t] = (float)H->Ci[l][t];
        }
    }
    H->have_f32 = 1;
    return ORC_OK;
}

/* Direct solve on the coarsest level: u_L = A_L^{-1} b_L with the band factor. */
static void coarse_solve_d(orc_hier *H)
{
    const int L = H->nlev - 1, nc = H->n[L];
    const size_t ld = (size_t)nc + 2;
    double *rhs = (double *)calloc((size_t)H->cm, sizeof(double));
    double *x = (double *)calloc((size_t)H->cm, sizeof(double));
    for (int j = 1; j <= nc; ++j)
        for (int i = 1; i <= nc; ++i) rhs[(i - 1) + nc * (j - 1)] = H->b[L][(size_t)j * ld + (size_t)i];
    orc_band_ldlt_solve(H->cm, H->cw, H->Lb, H->Db, rhs, x);
    for (int j = 1; j <= nc; ++j)
        for (int i = 1; i <= nc; ++i) H->u[L][(size_t)j * ld + (size_t)i] = x[(i - 1) + nc * (j - 1)];
    free(rhs);
    free(x);
}

/* The coarsest solve of the FP32 cycle stays in FP64: widen, solve, round. */
static void coarse_solve_f(orc_hier *H)
{
    const int L = H->nlev - 1, nc = H->n[L];
    const size_t ld = (size_t)nc + 2;
    double *rhs = (double *)calloc((size_t)H->cm, sizeof(double));
    double *x = (double *)calloc((size_t)H->cm, sizeof(double));
    for (int j = 1; j <= nc; ++j)
        for (int i = 1; i <= nc; ++i)
            rhs[(i - 1) + nc * (j - 1)] = (double)H->fb[L][(size_t)j * ld + (size_t)i];
    orc_band_ldlt_solve(H->cm, H->cw, H->Lb, H->Db, rhs, x);
    for (int j = 1; j <= nc; ++j)
        for (int i = 1; i <= nc; ++i) H->fu[L][(size_t)j * ld + (size_t)i] = (float)x[(i - 1) + nc * (j - 1)];
    free(rhs);
    free(x);
}

/* V(nu1,nu2) cycle from level l (Fig. vcycle_flowchart): relax, form the
 * residual, restrict it as the next right-hand side with a zero initial
 * guess, recurse, interpolate and correct, relax again; direct solve on the
 * coarsest level. */
static void vcycle_d(orc_hier *H, int l)
{
    if (l == H->nlev - 1) { coarse_solve_d(H); return; }
    const int n = H->n[l];
    relax_d(H, l, H->nu1);
    residual_d(n, H->O[l], H->W[l], H->S[l], H->SW[l], H->NW[l], H->b[l], H->u[l], H->r[l]);
    restrict__d(n, H->Ci[l], H->r[l], H->b[l + 1]);
    memset(H->u[l + 1], 0, (size_t)(H->n[l + 1] + 2) * (H->n[l + 1] + 2) * sizeof(double));
    vcycle_d(H, l + 1);
    interp_add_d(n, H->Ci[l], H->u[l + 1], H->u[l]);
    relax_d(H, l, H->nu2);
}

static void vcycle_f(orc_hier *H, int l)
{
    if (l == H->nlev - 1) { coarse_solve_f(H); return; }
    const int n = H->n[l];
    gs_sweeps_f(n, H->fO[l], H->fW[l], H->fS[l], H->fSW[l], H->fNW[l], H->fb[l], H->fu[l], H->nu1);
    residual_f(n, H->fO[l], H->fW[l], H->fS[l], H->fSW[l], H->fNW[l], H->fb[l], H->fu[l], H->fr[l]);
    restrict__f(n, H->fCi[l], H->fr[l], H->fb[l + 1]);
    memset(H->fu[l + 1], 0, (size_t)(H->n[l + 1] + 2) * (H->n[l + 1] + 2) * sizeof(float));
    vcycle_f(H, l + 1);
    interp_add_f(n, H->fCi[l], H->fu[l + 1], H->fu[l]);
    gs_sweeps_f(n, H->fO[l], H->fW[l], H->fS[l], H->fSW[l], H->fNW[l], H->fb[l], H->fu[l], H->nu2);
}

/* One V-cycle on the fine level: b, u are (n+2)^2 padded arrays; u in/out. */
void orc_vcycle(orc_hier *H, const double *b, double *u)
{
    const size_t sz = (size_t)(H->n[0] + 2) * (H->n[0] + 2);
    memcpy(H->b[0], b, sz * sizeof(double));
    memcpy(H->u[0], u, sz * sizeof(double));
    vcycle_d(H, 0);
    memcpy(u, H->u[0], sz * sizeof(double));
}

/* One level-l step, on the hierarchy's own arrays: 0 = nu relaxation sweeps
 * (point or line Gauss-Seidel as set; arg = sweeps), 1 = residual into r, 2 = restriction of r into b_{l+1} and zero
 * u_{l+1}, 3 = u += P u_{l+1}, 4 = coarsest direct solve. */
void orc_step(orc_hier *H, int l, int op, int arg)
{
    const int n = H->n[l];
    switch (op) {
    case 0: relax_d(H, l, arg); break;
    case 1: residual_d(n, H->O[l], H->W[l], H->S[l], H->SW[l], H->NW[l], H->b[l], H->u[l], H->r[l]); break;
    case 2:
        restrict__d(n, H->Ci[l], H->r[l], H->b[l + 1]);
        memset(H->u[l + 1], 0, (size_t)(H->n[l + 1] + 2) * (H->n[l + 1] + 2) * sizeof(double));
        break;
    case 3: interp_add_d(n, H->Ci[l], H->u[l + 1], H->u[l]); break;
    case 4: coarse_solve_d(H); break;
    default: break;
    }
}

/* Relative residual ||b - A (xh + xl)||_2 / ||b||_2 over the interior of
 * level 0, with the accurate residual (xl nullable). */
double orc_rel_residual(orc_hier *H, const double *b, const double *xh, const double *xl)
{
    const int n = H->n[0];
    residual_dd(n, H->O[0], H->W[0], H->S[0], H->SW[0], H->NW[0], b, xh, xl, H->r[0]);
    const double nr = orc_sumsq(n, H->r[0]);
    const double nb = orc_sumsq(n, b);
    return sqrt(nr) / sqrt(nb);
}

/* Solve to ||b - A x||_2/||b||_2 <= tol, checked after every cycle with the
 * accurate residual, or max_cycles.  V(nu1,nu2)-cycles on the FP64 iterate
 * until the relative residual is <= refine_factor * tol (refine_factor = 0:
 * never); from then on the iterate is carried as a double-FP64 pair
 * (xh, xl) and each cycle is one refinement step: r = b - A (xh + xl)
 * (accurate residual, rounded once), d = V(nu1,nu2)(0, r), (xh, xl) += d in
 * double-FP64.  In exact arithmetic both forms are the same iteration; the
 * second one keeps converging below the residual floor of FP64 vectors.
 * u: (n+2)^2 initial guess in, xh out; xl: (n+2)^2 out or NULL.
 * hist receives the relative residual after each cycle; returns the number of
 * cycles run.  ||b|| = 0 gives u = 0 after 0 cycles. */
int orc_solve(orc_hier *H, const double *b, double *u, double *xl_out, double tol,
              int max_cycles, int refine_factor, double *hist)
{
    const int n = H->n[0];
    const size_t sz = (size_t)(n + 2) * (n + 2);
    if (xl_out) memset(xl_out, 0, sz * sizeof(double));
    if (orc_sumsq(n, b) == 0.0) {
        memset(u, 0, sz * sizeof(double));
        return 0;
    }
    const double nb = sqrt(orc_sumsq(n, b));
    double *xl = (double *)calloc(sz, sizeof(double));
    double *r = (double *)calloc(sz, sizeof(double));
    memcpy(H->b[0], b, sz * sizeof(double));
    memcpy(H->u[0], u, sz * sizeof(double));
    int k = 0, phase = 0;
    while (k < max_cycles) {
        vcycle_d(H, 0);
        if (phase == 0) {
            residual_dd(n, H->O[0], H->W[0], H->S[0], H->SW[0], H->NW[0], b, H->u[0], NULL, r);
        } else {
            for (size_t t = 0; t < sz; ++t) dd_add(&u[t], &xl[t], H->u[0][t]);
            residual_dd(n, H->O[0], H->W[0], H->S[0], H->SW[0], H->NW[0], b, u, xl, r);
        }
        const double rho = sqrt(orc_sumsq(n, r)) / nb;
        if (hist) hist[k] = rho;
        ++k;
        if (!(rho > tol)) break;
        if (phase == 0 && refine_factor > 0 && rho <= refine_factor * tol) {
            phase = 1;
            memcpy(u, H->u[0], sz * sizeof(double));
        }
        if (phase == 1) {
            memcpy(H->b[0], r, sz * sizeof(double));
            memset(H->u[0], 0, sz * sizeof(double));
        }
    }
    if (phase == 0) memcpy(u, H->u[0], sz * sizeof(double));
    else if (xl_out) memcpy(xl_out, xl, sz * sizeof(double));
    free(xl);
    free(r);
    return k;
}

/* FP32 V-cycle (FP32-rounded hierarchy, FP64 coarsest solve) as the
 * preconditioner of iterative refinement on a double-FP64 iterate:
 *   (xh, xl) = (given, 0); loop: r = b - A (xh + xl) (accurate residual);
 *   rho = ||r||/||b||, stop if <= tol; s = the smallest power of two
 *   >= ||r||_inf; r32 = fl32(r / s); d32 = V32(nu1,nu2)(0, r32);
 *   (xh, xl) += s * d32 in double-FP64.
 * hist receives rho before each correction (hist[0] is the initial residual);
 * returns the number of corrections applied. */
int orc_solve_ir(orc_hier *H, const double *b, double *x, double *xl_out, double tol,
                 int max_iter, double *hist)
{
    const int n = H->n[0];
    const size_t ld = (size_t)n + 2, sz = ld * ld;
    orc_make_f32(H);
    if (xl_out) memset(xl_out, 0, sz * sizeof(double));
    const double nb = sqrt(orc_sumsq(n, b));
    if (nb == 0.0) { memset(x, 0, sz * sizeof(double)); return 0; }
    double *r = H->r[0];
    double *xl = (double *)calloc(sz, sizeof(double));
    int it = 0;
    for (;;) {
        residual_dd(n, H->O[0], H->W[0], H->S[0], H->SW[0], H->NW[0], b, x, xl, r);
        const double rho = sqrt(orc_sumsq(n, r)) / nb;
        if (hist) hist[it] = rho;
        if (!(rho > tol) || it >= max_iter) break;
        double rmax = 0.0;
        for (size_t t = 0; t < sz; ++t) {
            const double a = fabs(r[t]);
            if (a > rmax) rmax = a;
        }
        int e;
        const double fr = frexp(rmax, &e);      /* rmax = fr * 2^e, fr in [0.5,1) */
        if (fr == 0.5) e -= 1;                 /* exact power of two */
        const double s = ldexp(1.0, e), inv = ldexp(1.0, -e);
        for (size_t t = 0; t < sz; ++t) H->fb[0][t] = (float)(r[t] * inv);
        memset(H->fu[0], 0, sz * sizeof(float));
        vcycle_f(H, 0);
        for (size_t t = 0; t < sz; ++t) dd_add(&x[t], &xl[t], s * (double)H->fu[0][t]);
        ++it;
    }
    if (xl_out) memcpy(xl_out, xl, sz * sizeof(double));
    free(xl);
    return it;
}

/* -------------------------------------------------- nonsymmetric BoxMG */
#include "bmg_oracle_ns.c"
