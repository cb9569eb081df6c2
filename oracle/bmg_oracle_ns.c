/*
 * Nonsymmetric black-box multigrid (part of the CPU oracle; included at the
 * end of bmg_oracle.c, so it shares that file's helpers).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of the oracle.
 *
 * The paper's method (Section 2, Fig. vcycle_flowchart) belongs to the BoxMG
 * family, whose nonsymmetric variant the paper's references describe: the
 * interpolation P is induced by the operator A as in the symmetric case, the
 * restriction is the transpose of the interpolation induced by the transposed
 * operator, R = P~^T, and the coarse operator is the Petrov-Galerkin product
 * A_c = R A P.  The readings taken here:
 *
 *  - every level keeps all nine entries of each row (no symmetric storage):
 *    planes A[e], e = SW, S, SE, W, O, E, NW, N, NE, A[e][p] the coupling of
 *    row p to p + d(e), zero on the Dirichlet ring;
 *  - P's weights (8 planes, the layout of the symmetric oracle) are the
 *    symmetric formulas applied to the lumped rows of A; R's weights are the
 *    same formulas applied to the lumped rows of A^T, row p of A^T holding
 *    A^T(p, p + d) = A(p + d, p);
 *  - the restriction b_c = R r is the symmetric restriction (Fig.
 *    restrict_kernel's term order) with R's weights in place of P's;
 *  - A_c(I,J; d) = sum_p R(p; IJ) sum_q A(p, q) P(q; IJ + d), for all nine d,
 *    p over the 3x3 fine patch (rows south to north), q over p's neighbours
 *    SW..NE inside the support of the basis function IJ + d, both sums from
 *    zero, couplings to ring coarse points dropped;
 *  - four-colour Gauss-Seidel and the residual take the nine entries of the
 *    row in the order SW, S, SE, W, E, NW, N, NE (centre last in the
 *    residual), the order of the symmetric oracle;
 *  - the coarsest level (lexicographic unknowns, a band of half-bandwidth
 *    w = n_L + 1 on both sides of the diagonal) is factored as A = L D U with
 *    unit triangular L and U, column by column: D_k = a_kk, L_ik = a_ik / D_k,
 *    U_kj = a_kj / D_k, and a_ij <- a_ij - L_ik a_kj for k < i, j <= k + w
 *    (each entry takes its terms in increasing k); the solves are the column
 *    forms of the symmetric oracle, each update one fused multiply-add:
 *    y_i -= L_ij y_j (j increasing), z = y / D, x_i -= U_ik x_k (k
 *    decreasing).
 *
 * With a symmetric A the weights of P and R, the smoother and the residual
 * are those of the symmetric oracle to the bit; the coarse operators agree to
 * rounding (the symmetric oracle forms only five directions and mirrors the
 * rest).
 */

#define NS_NE 9
enum { NS_SW = 0, NS_S, NS_SE, NS_W, NS_O, NS_E, NS_NW, NS_N, NS_NEd };

/* offset of stencil entry e in a padded array of row length ld */
static ptrdiff_t ns_off(int e, size_t ld)
{
    return (ptrdiff_t)(e % 3 - 1) + (ptrdiff_t)(e / 3 - 1) * (ptrdiff_t)ld;
}

/* Row p of A (transpose = 0) or of A^T (transpose = 1). */
static void ns_row(double *const A[NS_NE], size_t ld, size_t p, int transpose, double a[NS_NE])
{
    for (int e = 0; e < NS_NE; ++e) {
        if (!transpose || e == NS_O) {
            a[e] = A[e][p];
        } else {
            /* A^T(p, p + d) = A(p + d, p): entry 8 - e of row p + d */
            a[e] = A[NS_NE - 1 - e][(size_t)((ptrdiff_t)p + ns_off(e, ld))];
        }
    }
}

/* Operator-induced weights of A (transpose = 0, the interpolation P) or of A^T
 * (transpose = 1, the weights whose transpose is the restriction): the
 * formulas of orc_interp_weights on the lumped rows.  Ci: 8 planes of
 * (nc+2)^2. */
int orc_ns_weights(int nf, double *const A[NS_NE], int transpose, double *Ci)
{
    if (!valid_n(nf) || nf < 7) return ORC_EINVAL;
    const int nc = (nf - 1) / 2;
    const size_t ldf = (size_t)nf + 2, ldc = (size_t)nc + 2, pl = ldc * ldc;
    double *LNE = Ci, *LA = Ci + pl, *LNW = Ci + 2 * pl, *LR = Ci + 3 * pl;
    double *LL = Ci + 4 * pl, *LSE = Ci + 5 * pl, *LB = Ci + 6 * pl, *LSW = Ci + 7 * pl;
    memset(Ci, 0, 8 * pl * sizeof(double));
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int J = 1; J <= nc + 1; ++J) {
        for (int I = 1; I <= nc + 1; ++I) {
            const size_t c = (size_t)J * ldc + (size_t)I;
            double a[NS_NE];
            if (J <= nc) {   /* x-edge (2I-1, 2J) */
                ns_row(A, ldf, (size_t)(2 * J) * ldf + (size_t)(2 * I - 1), transpose, a);
                lump9(a);
                const double D = (a[NS_O] + a[NS_N]) + a[NS_S];
                if (!(D > 0.0)) bad = 1;
                LL[c] = -((a[NS_W] + a[NS_NW]) + a[NS_SW]) / D;
                LR[c] = -((a[NS_E] + a[NS_NEd]) + a[NS_SE]) / D;
            }
            if (I <= nc) {   /* y-edge (2I, 2J-1) */
                ns_row(A, ldf, (size_t)(2 * J - 1) * ldf + (size_t)(2 * I), transpose, a);
                lump9(a);
                const double D = (a[NS_O] + a[NS_W]) + a[NS_E];
                if (!(D > 0.0)) bad = 1;
                LB[c] = -((a[NS_S] + a[NS_SW]) + a[NS_SE]) / D;
                LA[c] = -((a[NS_N] + a[NS_NW]) + a[NS_NEd]) / D;
            }
        }
    }
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int J = 1; J <= nc + 1; ++J) {
        for (int I = 1; I <= nc + 1; ++I) {
            const size_t c = (size_t)J * ldc + (size_t)I;
            double a[NS_NE];
            ns_row(A, ldf, (size_t)(2 * J - 1) * ldf + (size_t)(2 * I - 1), transpose, a);
            lump9(a);
            if (!(a[NS_O] > 0.0)) bad = 1;
            LNE[c] = -((a[NS_NEd] + a[NS_N] * LR[c]) + a[NS_E] * LA[c]) / a[NS_O];
            LNW[c] = -((a[NS_NW] + a[NS_N] * LL[c]) + a[NS_W] * LA[c - 1]) / a[NS_O];
            LSE[c] = -((a[NS_SE] + a[NS_S] * LR[c - ldc]) + a[NS_E] * LB[c]) / a[NS_O];
            LSW[c] = -((a[NS_SW] + a[NS_S] * LL[c - ldc]) + a[NS_W] * LB[c - 1]) / a[NS_O];
        }
    }
    return bad ? ORC_EBREAKDOWN : ORC_OK;
}

/* Petrov-Galerkin coarse operator A_c = R A P, all nine directions (see the
 * header), into the nine planes Ac of (nc+2)^2. */
int orc_ns_rap(int nf, double *const A[NS_NE], const double *Pi, const double *Ri, double *const Ac[NS_NE])
{
    if (!valid_n(nf) || nf < 7) return ORC_EINVAL;
    const int nc = (nf - 1) / 2;
    const size_t ldf = (size_t)nf + 2, ldc = (size_t)nc + 2, plc = ldc * ldc;
    for (int e = 0; e < NS_NE; ++e) memset(Ac[e], 0, plc * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int J = 1; J <= nc; ++J) {
        for (int I = 1; I <= nc; ++I) {
            for (int d = 0; d < NS_NE; ++d) {
                const int KI = I + d % 3 - 1, KJ = J + d / 3 - 1;
                double acc = 0.0;
                if (KI >= 1 && KI <= nc && KJ >= 1 && KJ <= nc) {
                    for (int jj = -1; jj <= 1; ++jj) {
                        for (int ii = -1; ii <= 1; ++ii) {
                            const int pi = 2 * I + ii, pj = 2 * J + jj;
                            const size_t p = (size_t)pj * ldf + (size_t)pi;
                            const double wp = pweight(Ri, ldc, I, J, pi, pj);
                            double a[NS_NE];
                            ns_row(A, ldf, p, 0, a);
                            double t = 0.0;
                            for (int e = 0; e < NS_NE; ++e) {
                                const int qi = pi + (e % 3) - 1, qj = pj + (e / 3) - 1;
                                if (abs(qi - 2 * KI) > 1 || abs(qj - 2 * KJ) > 1) continue;
                                t = t + a[e] * pweight(Pi, ldc, KI, KJ, qi, qj);
                            }
                            acc = acc + wp * t;
                        }
                    }
                }
                Ac[d][(size_t)J * ldc + (size_t)I] = acc;
            }
        }
    }
    return ORC_OK;
}

/* Four-colour Gauss-Seidel with full rows: per point s = b; s -= A_d u_d for
 * d = SW, S, SE, W, E, NW, N, NE; u = s / A_O. */
void orc_ns_gs(int n, double *const A[NS_NE], const double *b, double *u, int sweeps)
{
    const size_t ld = (size_t)n + 2;
    static const int order[8] = {NS_SW, NS_S, NS_SE, NS_W, NS_E, NS_NW, NS_N, NS_NEd};
    for (int sweep = 0; sweep < sweeps; ++sweep) {
        for (int c = 0; c < 4; ++c) {
            const int j0 = (c >> 1) ? 1 : 2, i0 = (c & 1) ? 1 : 2;
#pragma omp parallel for schedule(static)
            for (int j = j0; j <= n; j += 2) {
                for (int i = i0; i <= n; i += 2) {
                    const size_t p = (size_t)j * ld + (size_t)i;
                    double s = b[p];
                    for (int t = 0; t < 8; ++t) {
                        const int e = order[t];
                        s -= A[e][p] * u[(size_t)((ptrdiff_t)p + ns_off(e, ld))];
                    }
                    u[p] = s / A[NS_O][p];
                }
            }
        }
    }
}

/* Residual r = b - A u, the smoother's order with the centre term last. */
void orc_ns_residual(int n, double *const A[NS_NE], const double *b, const double *u, double *r)
{
    const size_t ld = (size_t)n + 2;
    static const int order[8] = {NS_SW, NS_S, NS_SE, NS_W, NS_E, NS_NW, NS_N, NS_NEd};
#pragma omp parallel for schedule(static)
    for (int j = 1; j <= n; ++j) {
        for (int i = 1; i <= n; ++i) {
            const size_t p = (size_t)j * ld + (size_t)i;
            double s = b[p];
            for (int t = 0; t < 8; ++t) {
                const int e = order[t];
                s -= A[e][p] * u[(size_t)((ptrdiff_t)p + ns_off(e, ld))];
            }
            s -= A[NS_O][p] * u[p];
            r[p] = s;
        }
    }
}

/* Band L D U factor of a nonsymmetric band matrix (m unknowns, w sub- and
 * super-diagonals), column by column as in the header.  Ab: row i holds
 * A_ik for k = i-w .. i+w at Ab[i (2w+1) + (k - i + w)] (zero outside the
 * matrix).  Lb[i w + (k - i + w)] = L_ik (k = i-w .. i-1), Ub[i w + (k - i - 1)]
 * = U_ik (k = i+1 .. i+w), D[i]. */
int orc_band_ldu_factor(int m, int w, const double *Ab, double *Lb, double *Ub, double *D)
{
    if (m < 1 || w < 1) return ORC_EINVAL;
    const size_t rw = 2 * (size_t)w + 1;
    double *a = (double *)malloc((size_t)m * rw * sizeof(double));
    if (!a) return ORC_ENOMEM;
    memcpy(a, Ab, (size_t)m * rw * sizeof(double));
    memset(Lb, 0, (size_t)m * (size_t)w * sizeof(double));
    memset(Ub, 0, (size_t)m * (size_t)w * sizeof(double));
#define AA(i, k) a[(size_t)(i) * rw + (size_t)((k) - (i) + w)]
    int st = ORC_OK;
    for (int k = 0; k < m && st == ORC_OK; ++k) {
        const double d = AA(k, k);
        if (!(d > 0.0)) st = ORC_EBREAKDOWN;
        D[k] = d;
        const int k1 = k + w < m - 1 ? k + w : m - 1;
        for (int i = k + 1; i <= k1; ++i) Lb[(size_t)i * w + (size_t)(k - i + w)] = AA(i, k) / d;
        for (int j = k + 1; j <= k1; ++j) Ub[(size_t)k * w + (size_t)(j - k - 1)] = AA(k, j) / d;
        for (int i = k + 1; i <= k1; ++i) {
            const double lik = Lb[(size_t)i * w + (size_t)(k - i + w)];
            for (int j = k + 1; j <= k1; ++j) AA(i, j) = AA(i, j) - lik * AA(k, j);
        }
    }
#undef AA
    free(a);
    return st;
}

/* x = U^-1 D^-1 L^-1 b, the column forms with fused updates (header). */
void orc_band_ldu_solve(int m, int w, const double *Lb, const double *Ub, const double *D, const double *b,
                        double *x)
{
    for (int i = 0; i < m; ++i) x[i] = b[i];
    for (int j = 0; j < m; ++j) {
        const int i1 = j + w < m - 1 ? j + w : m - 1;
        for (int i = j + 1; i <= i1; ++i) x[i] = fma(-Lb[(size_t)i * w + (size_t)(j - i + w)], x[j], x[i]);
    }
    for (int i = 0; i < m; ++i) x[i] = x[i] / D[i];
    for (int k = m - 1; k >= 0; --k) {
        for (int i = k - w > 0 ? k - w : 0; i < k; ++i)
            x[i] = fma(-Ub[(size_t)i * w + (size_t)(k - i - 1)], x[k], x[i]);
    }
}

/* ------------------------------------------------- hierarchy and solve */
typedef struct {
    int nlev, n[ORC_MAXL];
    double *A[ORC_MAXL][NS_NE];
    double *Pi[ORC_MAXL], *Ri[ORC_MAXL];   /* weights between level l and l+1 */
    double *u[ORC_MAXL], *b[ORC_MAXL], *r[ORC_MAXL];
    double *Lb, *Ub, *Db;                   /* coarsest band L D U */
    int cm, cw, nu1, nu2;
} orc_ns_hier;

void orc_ns_destroy(orc_ns_hier *H)
{
    if (!H) return;
    for (int l = 0; l < ORC_MAXL; ++l) {
        for (int e = 0; e < NS_NE; ++e) free(H->A[l][e]);
        free(H->Pi[l]); free(H->Ri[l]); free(H->u[l]); free(H->b[l]); free(H->r[l]);
    }
    free(H->Lb); free(H->Ub); free(H->Db);
    free(H);
}

/* Hierarchy of a [n][n][K] stencil (K = 5: S, W, O, E, N; K = 9: SW .. NE),
 * levels down to `coarsest` points per side. */
orc_ns_hier *orc_ns_setup(int n, int K, const double *stencil, int nu1, int nu2, int coarsest, int *status)
{
    *status = ORC_EINVAL;
    if (!valid_n(n) || (K != 5 && K != 9) || !valid_n(coarsest) || coarsest > n || coarsest > 63) return NULL;
    orc_ns_hier *H = (orc_ns_hier *)calloc(1, sizeof(orc_ns_hier));
    H->nu1 = nu1;
    H->nu2 = nu2;
    int nl = 0;
    for (int m = n; m >= coarsest && nl < ORC_MAXL; m = (m - 1) / 2) H->n[nl++] = m;
    H->nlev = nl;
    for (int l = 0; l < nl; ++l) {
        const size_t sz = (size_t)(H->n[l] + 2) * (H->n[l] + 2);
        for (int e = 0; e < NS_NE; ++e) H->A[l][e] = zalloc(sz);
        H->u[l] = zalloc(sz); H->b[l] = zalloc(sz); H->r[l] = zalloc(sz);
        if (l + 1 < nl) {
            const size_t szc = (size_t)(H->n[l + 1] + 2) * (H->n[l + 1] + 2);
            H->Pi[l] = zalloc(8 * szc);
            H->Ri[l] = zalloc(8 * szc);
        }
    }
    /* level 0 from the stencil: entries to the ring must be zero */
    static const int map5[5] = {NS_S, NS_W, NS_O, NS_E, NS_N};
    const size_t ld = (size_t)n + 2;
    for (int j = 1; j <= n; ++j) {
        for (int i = 1; i <= n; ++i) {
            const double *q = stencil + ((size_t)(j - 1) * n + (size_t)(i - 1)) * (size_t)K;
            const size_t p = (size_t)j * ld + (size_t)i;
            for (int t = 0; t < K; ++t) {
                const int e = K == 5 ? map5[t] : t;
                const int qi = i + e % 3 - 1, qj = j + e / 3 - 1;
                if (e != NS_O && (qi < 1 || qi > n || qj < 1 || qj > n) && q[t] != 0.0) {
                    orc_ns_destroy(H);
                    return NULL;
                }
                H->A[0][e][p] = q[t];
            }
        }
    }
    for (int l = 0; l + 1 < nl; ++l) {
        int s1 = orc_ns_weights(H->n[l], H->A[l], 0, H->Pi[l]);
        int s2 = orc_ns_weights(H->n[l], H->A[l], 1, H->Ri[l]);
        if (s1 || s2) { *status = ORC_EBREAKDOWN; orc_ns_destroy(H); return NULL; }
        orc_ns_rap(H->n[l], H->A[l], H->Pi[l], H->Ri[l], H->A[l + 1]);
    }
    /* coarsest band L D U */
    const int nc = H->n[nl - 1], m = nc * nc, w = nc + 1;
    const size_t ldc = (size_t)nc + 2, rw = 2 * (size_t)w + 1;
    double *Ab = zalloc((size_t)m * rw);
    for (int j = 1; j <= nc; ++j) {
        for (int i = 1; i <= nc; ++i) {
            const int k = (i - 1) + nc * (j - 1);
            for (int e = 0; e < NS_NE; ++e) {
                const int qi = i + e % 3 - 1, qj = j + e / 3 - 1;
                if (qi < 1 || qi > nc || qj < 1 || qj > nc) continue;
                const int q = (qi - 1) + nc * (qj - 1);
                Ab[(size_t)k * rw + (size_t)(q - k + w)] = H->A[nl - 1][e][(size_t)j * ldc + (size_t)i];
            }
        }
    }
    H->cm = m;
    H->cw = w;
    H->Lb = zalloc((size_t)m * w);
    H->Ub = zalloc((size_t)m * w);
    H->Db = zalloc((size_t)m);
    const int sf = orc_band_ldu_factor(m, w, Ab, H->Lb, H->Ub, H->Db);
    free(Ab);
    if (sf) { *status = sf; orc_ns_destroy(H); return NULL; }
    *status = ORC_OK;
    return H;
}

int orc_ns_num_levels(const orc_ns_hier *H) { return H->nlev; }
int orc_ns_level_n(const orc_ns_hier *H, int l) { return H->n[l]; }

/* Level arrays: 0..8 the stencil planes, 9 P's weights, 10 R's weights,
 * 11 u, 12 b, 13 r. */
double *orc_ns_field(orc_ns_hier *H, int l, int f)
{
    if (l < 0 || l >= H->nlev) return NULL;
    if (f >= 0 && f < NS_NE) return H->A[l][f];
    switch (f) {
    case 9: return H->Pi[l];
    case 10: return H->Ri[l];
    case 11: return H->u[l];
    case 12: return H->b[l];
    case 13: return H->r[l];
    default: return NULL;
    }
}

/* The coarsest factor: m w entries of L, m w of U, m of D; sizes if NULL. */
void orc_ns_coarse_factor(const orc_ns_hier *H, double *Lb, double *Ub, double *D, int *m, int *w)
{
    if (m) *m = H->cm;
    if (w) *w = H->cw;
    if (Lb) memcpy(Lb, H->Lb, (size_t)H->cm * H->cw * sizeof(double));
    if (Ub) memcpy(Ub, H->Ub, (size_t)H->cm * H->cw * sizeof(double));
    if (D) memcpy(D, H->Db, (size_t)H->cm * sizeof(double));
}

static void ns_coarse_solve(orc_ns_hier *H)
{
    const int L = H->nlev - 1, nc = H->n[L];
    const size_t ld = (size_t)nc + 2;
    double *rhs = zalloc((size_t)H->cm), *x = zalloc((size_t)H->cm);
    for (int j = 1; j <= nc; ++j)
        for (int i = 1; i <= nc; ++i) rhs[(i - 1) + nc * (j - 1)] = H->b[L][(size_t)j * ld + (size_t)i];
    orc_band_ldu_solve(H->cm, H->cw, H->Lb, H->Ub, H->Db, rhs, x);
    for (int j = 1; j <= nc; ++j)
        for (int i = 1; i <= nc; ++i) H->u[L][(size_t)j * ld + (size_t)i] = x[(i - 1) + nc * (j - 1)];
    free(rhs);
    free(x);
}

/* V(nu1,nu2) cycle from level l, as the symmetric one with R restricting. */
static void ns_vcycle(orc_ns_hier *H, int l)
{
    if (l == H->nlev - 1) { ns_coarse_solve(H); return; }
    const int n = H->n[l];
    orc_ns_gs(n, H->A[l], H->b[l], H->u[l], H->nu1);
    orc_ns_residual(n, H->A[l], H->b[l], H->u[l], H->r[l]);
    restrict__d(n, H->Ri[l], H->r[l], H->b[l + 1]);
    memset(H->u[l + 1], 0, (size_t)(H->n[l + 1] + 2) * (H->n[l + 1] + 2) * sizeof(double));
    ns_vcycle(H, l + 1);
    interp_add_d(n, H->Pi[l], H->u[l + 1], H->u[l]);
    orc_ns_gs(n, H->A[l], H->b[l], H->u[l], H->nu2);
}

/* One level-l step on the hierarchy's arrays: 0 = arg sweeps, 1 = residual,
 * 2 = restriction into b_{l+1} (u_{l+1} zeroed), 3 = u += P u_{l+1},
 * 4 = coarsest solve. */
void orc_ns_step(orc_ns_hier *H, int l, int op, int arg)
{
    const int n = H->n[l];
    switch (op) {
    case 0: orc_ns_gs(n, H->A[l], H->b[l], H->u[l], arg); break;
    case 1: orc_ns_residual(n, H->A[l], H->b[l], H->u[l], H->r[l]); break;
    case 2:
        restrict__d(n, H->Ri[l], H->r[l], H->b[l + 1]);
        memset(H->u[l + 1], 0, (size_t)(H->n[l + 1] + 2) * (H->n[l + 1] + 2) * sizeof(double));
        break;
    case 3: interp_add_d(n, H->Pi[l], H->u[l + 1], H->u[l]); break;
    case 4: ns_coarse_solve(H); break;
    default: break;
    }
}

/* V-cycles from u until ||b - A u||_2 / ||b||_2 <= tol (checked after every
 * cycle, the sum of squares accurately rounded) or max_cycles; hist[k] is the
 * relative residual after cycle k+1.  Returns the number of cycles. */
int orc_ns_solve(orc_ns_hier *H, const double *b, double *u, double tol, int max_cycles, double *hist)
{
    const int n = H->n[0];
    const size_t sz = (size_t)(n + 2) * (n + 2);
    const double nb = sqrt(orc_sumsq(n, b));
    if (nb == 0.0) { memset(u, 0, sz * sizeof(double)); return 0; }
    memcpy(H->b[0], b, sz * sizeof(double));
    memcpy(H->u[0], u, sz * sizeof(double));
    int k = 0;
    while (k < max_cycles) {
        ns_vcycle(H, 0);
        orc_ns_residual(n, H->A[0], b, H->u[0], H->r[0]);
        const double rho = sqrt(orc_sumsq(n, H->r[0])) / nb;
        if (hist) hist[k] = rho;
        ++k;
        if (!(rho > tol)) break;
    }
    memcpy(u, H->u[0], sz * sizeof(double));
    return k;
}
