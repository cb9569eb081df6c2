// Host side of the black-box multigrid library: workspace planning, set-up,
// the V-cycle driver, the solve loop and the C entry points of bmg.h.
//
// One level hierarchy lives in the caller's workspace; nothing here calls
// hipMalloc.  Every launch goes to the handle's stream.
#include "bmg_internal.hpp"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

using namespace bmgi;

namespace bmgi {

thread_local char g_err[512];

bmg_status fail(bmg_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

// Tile rows chosen by the autotuner, per level size n = 2^m - 1 (0 = unset).
static int g_tile_rows[17];

int tile_rows_for(const bmg_solver *h, int n, bool nine)
{
    if (h && h->opt.tile_rows > 0) return h->opt.tile_rows;
    int m = 0;
    while ((1 << m) < n + 1 && m < 16) ++m;
    if (g_tile_rows[m] > 0) return g_tile_rows[m];
    // measured defaults (FP64, V(2,1)): the fewest warm-up rows re-read while
    // the tiles still fill the chip in whole rounds (at 4095^2, 96 rows give
    // 731 tiles, one round of three 48 KiB pre-pass or four 40 KiB post-pass
    // workgroups per CU, where 64 rows give 1088 and a second round of 64, and
    // a second round costs more than the rows it saves); on the levels below 1023 the
    // shortest tiles win, their passes being bound by the latency of the row
    // pipeline rather than by bandwidth
    // at 8191^2 (the FP32 refinement's fine level, five 20 KiB workgroups
    // per CU) 224 rows give 1258 tiles, one round of 1280
    if (n >= 8191) return 224;
    if (n >= 4095) return 96;
    // nine-point tiles take 72 KiB of LDS, two per CU: 40 rows give 468
    // tiles at 2047^2 and 12 rows 430 at 1023^2, each one round of 512 (36
    // and 10 rows give 513 and 515)
    if (n >= 2047) return nine ? 40 : 48;
    if (n >= 1023) return nine ? 12 : 16;
    if (n >= 511) return 4;
    return 2;
}

TileGeo tile_geo(int n, int hx, int ht)
{
    TileGeo g;
    g.hx = hx;
    g.ht = std::max(2, std::min(ht, (n + 2) & ~1));
    const int useful = FW - 2 * hx;
    g.tiles_x = (n + useful - 1) / useful;
    g.ntiles = g.tiles_x * ((n + g.ht - 1) / g.ht);
    return g;
}

}  // namespace bmgi

extern "C" bmg_status bmg_tile_rows_set(int n, int rows)
{
    if (!valid_n(n)) return fail(BMG_EINVAL, "n=%d is not 2^m-1", n);
    if (rows < 0 || (rows & 1) || rows > 65536) return fail(BMG_EINVAL, "rows=%d must be even, 0 = default", rows);
    int m = 0;
    while ((1 << m) < n + 1) ++m;
    g_tile_rows[m] = rows;
    return BMG_OK;
}

extern "C" bmg_status bmg_tile_rows_get(int n, int *rows)
{
    if (!valid_n(n) || !rows) return fail(BMG_EINVAL, "bad arguments");
    *rows = tile_rows_for(nullptr, n, false);
    return BMG_OK;
}

namespace {

enum { S_SUMSQ = 0, S_BNORM = 1, S_REL0 = 2, S_TMP = 3, S_RMAX = 4, S_SCALE = 5, S_FLOOR = 6, S_NSCAL = 8 };

int coarsest_of(const bmg_options &o) { return o.coarsest_n > 0 ? o.coarsest_n : 3; }

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}
int persistent_of(const bmg_options &o) { return o.persistent_below_n > 0 ? o.persistent_below_n : SMALL_MAX_N; }
// Fused passes of level l in square tiles (k_pre2d, k_post2d)?
static bool square_tiles(const bmg_solver *h, int l)
{
    const int lim = h->opt.square_tiles_below_n > 0 ? h->opt.square_tiles_below_n : T2D_MAX_N;
    return h->nine[l] && h->nrhs == 1 && h->L[l].n <= lim;
}

// Walks the workspace layout; with base == nullptr it only measures.
size_t plan(bmg_solver *h, int n, int kind, const bmg_options &o, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + ALIGN - 1) & ~(ALIGN - 1);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    int nl = 0, ns[MAXL];
    const int ncoarse = coarsest_of(o);
    for (int m = n; m >= ncoarse && nl < MAXL; m = (m - 1) / 2) ns[nl++] = m;
    const bool f32 = o.precision == BMG_FP32_IR;
    for (int l = 0; l < nl; ++l) {
        const int ld = pitch_of(ns[l]);
        const size_t pl = (size_t)(ns[l] + 2) * ld;
        const bool nine = l > 0 || kind == 9;
        Lev<double> D{};
        D.n = ns[l];
        D.ld = ld;
        double *ua = (double *)take(pl * 8);
        D.u = (double *)take(pl * 8);
        D.b = (double *)take(pl * 8);
        D.r = (double *)take(pl * 8);
        D.O = (double *)take(pl * 8);
        D.W = (double *)take(pl * 8);
        D.S = (double *)take(pl * 8);
        D.SW = nine ? (double *)take(pl * 8) : nullptr;
        D.NW = nine ? (double *)take(pl * 8) : nullptr;
        Wts<double> W{};
        if (l + 1 < nl) {
            const int ldc = pitch_of(ns[l + 1]);
            W.ld = ldc;
            W.ps = (size_t)(ns[l + 1] + 2) * ldc;
            W.p = (double *)take(8 * W.ps * 8);
        }
        Lev<float> F{};
        Wts<float> FW{};
        float *ua32 = nullptr;
        if (f32) {
            F.n = ns[l];
            F.ld = ld;
            ua32 = (float *)take(pl * 4);
            F.u = (float *)take(pl * 4);
            F.b = (float *)take(pl * 4);
            F.r = (float *)take(pl * 4);
            F.O = (float *)take(pl * 4);
            F.W = (float *)take(pl * 4);
            F.S = (float *)take(pl * 4);
            F.SW = nine ? (float *)take(pl * 4) : nullptr;
            F.NW = nine ? (float *)take(pl * 4) : nullptr;
            if (l + 1 < nl) {
                FW.ld = W.ld;
                FW.ps = W.ps;
                FW.p = (float *)take(8 * W.ps * 4);
            }
        }
        double *lf[5] = {};
        if (o.smoother == BMG_SMOOTH_LINE)
            for (int q = 0; q < 5; ++q) lf[q] = (double *)take(pl * 8);
        if (h) {
            h->lfy[l] = lf[0];
            h->rfy[l] = lf[1];
            h->lfx[l] = lf[2];
            h->rfx[l] = lf[3];
            h->WT[l] = lf[4];
            h->L[l] = D;
            h->C[l] = W;
            h->nine[l] = nine;
            h->L32[l] = F;
            h->C32[l] = FW;
            h->ualt[l] = ua;
            h->ualt32[l] = ua32;
        }
    }
    const size_t pl0 = (size_t)(ns[0] + 2) * pitch_of(ns[0]);
    double *lineD = o.smoother == BMG_SMOOTH_LINE ? (double *)take(pl0 * 8) : nullptr;
    double *B0 = (double *)take(pl0 * 8);
    double *XH = (double *)take(pl0 * 8);
    double *XL = (double *)take(pl0 * 8);
    // coarsest factor: band storage of L and D (one block, for export), and
    // the rows of the one-wave solve
    const int cm = ns[nl - 1] * ns[nl - 1], cw = ns[nl - 1] + 1, cM = band_padded(cm);
    double *Lb = (double *)take(((size_t)cm * cw + cm) * 8);
    double *CF = (double *)take((size_t)cM * 64 * 8);
    double *CG = (double *)take((size_t)cM * 64 * 8);
    double *Dp = (double *)take((size_t)cM * 8);
    int *flags = (int *)take(64);
    double *part = (double *)take(NPART * 8);
    double *scal = (double *)take(S_NSCAL * 8);
    const int cap = std::max(o.max_cycles, 1) + 2;
    double *hist = (double *)take((size_t)cap * 8);
    int *cnt = (int *)take(64);
    if (h) {
        h->nlev = nl;
        h->lineD = lineD;
        h->B0 = B0;
        h->XH = XH;
        h->XL = XL;
        h->Lb = Lb;
        h->Dd = Lb + (size_t)cm * cw;
        h->band.CF = CF;
        h->band.CG = CG;
        h->band.Dp = Dp;
        h->band.m = cm;
        h->band.M = cM;
        h->band.nc = ns[nl - 1];
        h->flags = flags;
        h->part = part;
        h->scal = scal;
        h->hist = hist;
        h->hist_cap = cap;
        h->count = cnt;
        h->stop = cnt + 1;
        h->f32 = f32;
    }
    return (off + ALIGN - 1) & ~(ALIGN - 1);
}

bmg_status check_options(const bmg_options &o)
{
    if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 < 1 || o.nu1 > 64 || o.nu2 > 64)
        return fail(BMG_EINVAL, "nu1=%d nu2=%d out of range", o.nu1, o.nu2);
    if (o.max_cycles < 1 || o.max_cycles > 1000000)
        return fail(BMG_EINVAL, "max_cycles=%d out of range", o.max_cycles);
    if (o.precision != BMG_FP64 && o.precision != BMG_FP32_IR)
        return fail(BMG_EINVAL, "unknown precision %d", o.precision);
    if (o.kernels != BMG_KERNELS_BASIC && o.kernels != BMG_KERNELS_FUSED)
        return fail(BMG_EINVAL, "unknown kernel path %d", o.kernels);
    if (o.check_every < 1 || o.check_every > 4096)
        return fail(BMG_EINVAL, "check_every=%d out of range", o.check_every);
    if (o.refine_factor < 0)
        return fail(BMG_EINVAL, "refine_factor=%d must be >= 0", o.refine_factor);
    if (o.tile_rows < 0 || (o.tile_rows & 1) || o.tile_rows > 65536)
        return fail(BMG_EINVAL, "tile_rows=%d must be even and in [0, 65536]", o.tile_rows);
    if (o.interp != BMG_INTERP_BOXMG && o.interp != BMG_INTERP_LEARNED)
        return fail(BMG_EINVAL, "unknown interpolation %d", o.interp);
    if (o.interp == BMG_INTERP_LEARNED && !o.net) return fail(BMG_EINVAL, "learned interpolation without a network");
    if (o.learned_levels < 0) return fail(BMG_EINVAL, "learned_levels=%d must be >= 0", o.learned_levels);
    if (o.smoother != BMG_SMOOTH_POINT && o.smoother != BMG_SMOOTH_LINE)
        return fail(BMG_EINVAL, "unknown smoother %d", o.smoother);
    if (o.smoother == BMG_SMOOTH_LINE && o.precision != BMG_FP64)
        return fail(BMG_EINVAL, "line relaxation runs FP64 hierarchies");
    if (o.coarsest_n != 0 && (!valid_n(o.coarsest_n) || o.coarsest_n > BAND_MAX_NC))
        return fail(BMG_EINVAL, "coarsest_n=%d must be 2^k-1 in [3, %d] (0 = 3)", o.coarsest_n, BAND_MAX_NC);
    if (o.persistent_below_n != 0 && o.persistent_below_n != 1 &&
        (!valid_n(o.persistent_below_n) || o.persistent_below_n > SMALL_MAX_N))
        return fail(BMG_EINVAL, "persistent_below_n=%d must be 2^k-1 <= %d, 1 (none) or 0 (= %d)",
                    o.persistent_below_n, SMALL_MAX_N, SMALL_MAX_N);
    if (o.graph_mode != 0 && o.graph_mode != 1) return fail(BMG_EINVAL, "graph_mode=%d must be 0 or 1", o.graph_mode);
    if (o.square_tiles_below_n != 0 && o.square_tiles_below_n != 1 && !valid_n(o.square_tiles_below_n))
        return fail(BMG_EINVAL, "square_tiles_below_n=%d must be 2^k-1, 1 (none) or 0 (= %d)",
                    o.square_tiles_below_n, T2D_MAX_N);
    return BMG_OK;
}

// ------------------------------------------------------------ tracing
// `bytes`: the algorithmic bytes of the bracketed launches (each array the
// kernels need read or written once), summed for bmg_trace_read.
void trace_begin(bmg_solver *h, int kclass, int level, double bytes)
{
    if (h->tr_class != kclass || h->tr_level != level) return;
    h->tr_pending = bytes;
    if (h->tr_used + 2 > (int)h->tr_ev.size()) {
        if ((int)h->tr_ev.size() >= 2 * MAX_TRACE) return;
        const size_t grow = std::min<size_t>(2 * MAX_TRACE, std::max<size_t>(64, 2 * h->tr_ev.size()));
        size_t old = h->tr_ev.size();
        h->tr_ev.resize(grow);
        for (size_t t = old; t < grow; ++t) (void)hipEventCreate(&h->tr_ev[t]);
    }
    (void)hipEventRecord(h->tr_ev[h->tr_used], h->st);
}

void trace_end(bmg_solver *h, int kclass, int level)
{
    if (h->tr_class != kclass || h->tr_level != level) return;
    if (h->tr_used + 2 > (int)h->tr_ev.size()) return;
    (void)hipEventRecord(h->tr_ev[h->tr_used + 1], h->st);
    h->tr_used += 2;
    h->tr_bytes += h->tr_pending;
}

// Elements of the stencil planes stored per point: O, W, S (five-point) or
// also SW, NW (nine-point).
static inline double stencil_planes(bool nine) { return nine ? 5.0 : 3.0; }

// -------------------------------------------------------- cycle steps
const dim3 B2(64, 4);

// `sweeps` alternating zebra line relaxations of level l (FP64).
bmg_status line_smooth(bmg_solver *h, const Lev<double> &L, bool nine, int sweeps, const int *stop, int l)
{
    const int n = L.n, ld = L.ld;
    const dim3 tb(LT, 8), tg((n + 2 + LT - 1) / LT, (n + 2 + LT - 1) / LT);
    double *D = h->lineD;
    // per relaxation and direction: b, u, the line coupling, the off-line
    // couplings (S or W; also SW, NW) and the factor l, r read, u written
    trace_begin(h, BMG_TRACE_SMOOTH, l, sweeps * 2.0 * 8.0 * (nine ? 9.0 : 7.0) * (double)n * n);
    for (int s = 0; s < sweeps; ++s) {
        for (int par = 1; par >= 0; --par) {   // x-lines: odd rows, then even
            const int nl = par ? (n + 1) / 2 : (n - 1) / 2;
            if (nine) hipLaunchKernelGGL((k_line_rhs_x<true>), tg, tb, 0, h->st, L, par, D, stop);
            else hipLaunchKernelGGL((k_line_rhs_x<false>), tg, tb, 0, h->st, L, par, D, stop);
            hipLaunchKernelGGL(k_line_solve, dim3((nl + LINE_G - 1) / LINE_G), dim3(64), 0, h->st, n, ld, par, D,
                               (const double *)h->lfx[l], (const double *)h->rfx[l], (const double *)h->WT[l], D,
                               stop);
            hipLaunchKernelGGL(k_line_put_x, tg, tb, 0, h->st, n, ld, par, (const double *)D, L.u, stop);
        }
        for (int par = 1; par >= 0; --par) {   // y-lines: odd columns, then even
            const int nl = par ? (n + 1) / 2 : (n - 1) / 2;
            const dim3 rb(64, 4), rg((nl + 63) / 64, (n + 3) / 4);
            if (nine) hipLaunchKernelGGL((k_line_rhs_y<true>), rg, rb, 0, h->st, L, par, D, stop);
            else hipLaunchKernelGGL((k_line_rhs_y<false>), rg, rb, 0, h->st, L, par, D, stop);
            hipLaunchKernelGGL(k_line_solve, dim3((nl + LINE_G - 1) / LINE_G), dim3(64), 0, h->st, n, ld, par, D,
                               (const double *)h->lfy[l], (const double *)h->rfy[l], (const double *)L.S, L.u,
                               stop);
        }
    }
    trace_end(h, BMG_TRACE_SMOOTH, l);
    LAUNCHCHK();
    return BMG_OK;
}

template <typename T>
bmg_status smooth(bmg_solver *h, const Lev<T> &L, bool nine, int sweeps, const int *stop, int level)
{
    if (sweeps <= 0) return BMG_OK;
    if constexpr (std::is_same<T, double>::value) {
        if (h->opt.smoother == BMG_SMOOTH_LINE) return line_smooth(h, L, nine, sweeps, stop, level);
    }
    // per sweep: stencil, b and u read, u written
    trace_begin(h, BMG_TRACE_SMOOTH, level,
                sweeps * (stencil_planes(nine) + 3.0) * sizeof(T) * (double)L.n * L.n);
    for (int s = 0; s < sweeps; ++s) {
        for (int c = 0; c < 4; ++c) {
            const int ni = (c & 1) ? (L.n + 1) / 2 : (L.n - 1) / 2;
            const int nj = (c >> 1) ? (L.n + 1) / 2 : (L.n - 1) / 2;
            const dim3 g = grid2(ni, nj, B2);
            if (nine) hipLaunchKernelGGL((k_gs_colour<T, true>), g, B2, 0, h->st, L, c, stop);
            else hipLaunchKernelGGL((k_gs_colour<T, false>), g, B2, 0, h->st, L, c, stop);
        }
    }
    trace_end(h, BMG_TRACE_SMOOTH, level);
    LAUNCHCHK();
    return BMG_OK;
}

template <typename T>
bmg_status residual(bmg_solver *h, const Lev<T> &L, bool nine, const int *stop)
{
    const dim3 g = grid2(L.n, L.n, B2);
    if (nine) hipLaunchKernelGGL((k_residual<T, true>), g, B2, 0, h->st, L, stop);
    else hipLaunchKernelGGL((k_residual<T, false>), g, B2, 0, h->st, L, stop);
    LAUNCHCHK();
    return BMG_OK;
}

template <typename T>
bmg_status restrict_(bmg_solver *h, const Lev<T> &F, const Wts<T> &C, const Lev<T> &Cl, const int *stop)
{
    hipLaunchKernelGGL((k_restrict<T>), grid2(Cl.n, Cl.n, B2), B2, 0, h->st, F.r, F.ld, C, Cl, stop);
    LAUNCHCHK();
    return BMG_OK;
}

template <typename T>
bmg_status interp(bmg_solver *h, const Lev<T> &F, const Wts<T> &C, const Lev<T> &Cl, const int *stop)
{
    launch_interp_add<T>(F, C, (const T *)Cl.u, stop, h->st);
    LAUNCHCHK();
    return BMG_OK;
}

template <typename T>
bmg_status coarse(bmg_solver *h, const Lev<T> &Cl, const int *stop)
{
    static bool attr_set[2] = {false, false};
    const int which = sizeof(T) == 8 ? 0 : 1;
    if (!attr_set[which]) {
        HIPCHK(hipFuncSetAttribute((const void *)k_coarse_solve<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)band_solve_lds(band_padded(BAND_MAX_NC * BAND_MAX_NC))));
        attr_set[which] = true;
    }
    hipLaunchKernelGGL((k_coarse_solve<T>), dim3(h->nrhs), dim3(BAND_SOLVE_THREADS), band_solve_lds(h->band.M), h->st,
                       Cl, h->band, h->ks[h->nlev - 1], stop, h->kstop);
    LAUNCHCHK();
    return BMG_OK;
}

template <typename T>
const Lev<T> &lev(const bmg_solver *h, int l);
template <>
const Lev<double> &lev<double>(const bmg_solver *h, int l) { return h->L[l]; }
template <>
const Lev<float> &lev<float>(const bmg_solver *h, int l) { return h->L32[l]; }
template <typename T>
const Wts<T> &wts(const bmg_solver *h, int l);
template <>
const Wts<double> &wts<double>(const bmg_solver *h, int l) { return h->C[l]; }
template <>
const Wts<float> &wts<float>(const bmg_solver *h, int l) { return h->C32[l]; }


// V(nu1,nu2) from level l down to the coarsest direct solve and back.
template <typename T>
bmg_status vcycle_from(bmg_solver *h, int l, const int *stop)
{
    const Lev<T> &F = lev<T>(h, l);
    if (l == h->nlev - 1) return coarse<T>(h, F, stop);
    const Lev<T> &Cl = lev<T>(h, l + 1);
    const Wts<T> &C = wts<T>(h, l);
    TRY(smooth<T>(h, F, h->nine[l], h->opt.nu1, stop, l));
    TRY(residual<T>(h, F, h->nine[l], stop));
    TRY(restrict_<T>(h, F, C, Cl, stop));
    TRY(vcycle_from<T>(h, l + 1, stop));
    TRY(interp<T>(h, F, C, Cl, stop));
    TRY(smooth<T>(h, F, h->nine[l], h->opt.nu2, stop, l));
    return BMG_OK;
}

// ------------------------------------------------------- fused passes
template <typename T>
Lev<T> &levm(bmg_solver *h, int l);
template <>
Lev<double> &levm<double>(bmg_solver *h, int l) { return h->L[l]; }
template <>
Lev<float> &levm<float>(bmg_solver *h, int l) { return h->L32[l]; }
template <typename T>
T *&ualt(bmg_solver *h, int l);
template <>
double *&ualt<double>(bmg_solver *h, int l) { return h->ualt[l]; }
template <>
float *&ualt<float>(bmg_solver *h, int l) { return h->ualt32[l]; }

int level_tile_rows(const bmg_solver *h, int l) { return tile_rows_for(h, h->L[l].n, h->nine[l]); }

dim3 tile_grid(const TileGeo &g) { return dim3(((g.ntiles * g.nrhs + 7) / 8) * 8); }

// The tiles of level l of every right-hand side of the handle.
TileGeo level_tiles(const bmg_solver *h, int l, int hx)
{
    TileGeo g = tile_geo(h->L[l].n, hx, level_tile_rows(h, l));
    g.nrhs = h->nrhs;
    g.kstop = h->kstop;
    g.kpart = h->kpart;
    g.ksf = h->ks[l];
    g.ksc = l + 1 < h->nlev ? h->ks[l + 1] : 0;
    return g;
}

// FP64 pre passes compute the restriction weights (1) or read them (0).
#ifndef BMG_PRE_WEIGHTS_IN_PASS
#define BMG_PRE_WEIGHTS_IN_PASS 1
#endif

template <typename T>
static bool pre_weights_in_pass(const bmg_solver *h, int l, bool nine)
{
    const bool learned = h->opt.interp == BMG_INTERP_LEARNED &&
                         (h->opt.learned_levels == 0 || l < h->opt.learned_levels);
    // with several right-hand sides the weight rows are shared through L2,
    // while computing them would repeat the divisions for each
    return BMG_PRE_WEIGHTS_IN_PASS && std::is_same<T, double>::value && !nine && !learned && h->nrhs == 1;
}

// Rows per step of the fused passes on five-point levels: 4 (k_pre4, k_post4)
// or 2 (the general k_pre, k_post).
#ifndef BMG_FIVE_POINT_STEP_ROWS
#define BMG_FIVE_POINT_STEP_ROWS 2
#endif

// nu sweeps, residual and restriction in one pass (results as SMOOTH,
// RESIDUAL, RESTRICT in turn); the level's iterate moves to the other buffer.
template <typename T>
bmg_status fused_pre(bmg_solver *h, int l, int nu, const int *stop)
{
    Lev<T> &F = levm<T>(h, l);
    const Lev<T> &Cl = lev<T>(h, l + 1);
    const Wts<T> &C = wts<T>(h, l);
    const bool nine = h->nine[l];
    if (nu < 1 || nu > 3) {
        TRY(smooth<T>(h, F, nine, nu, stop, l));
        TRY(residual<T>(h, F, nine, stop));
        return restrict_<T>(h, F, C, Cl, stop);
    }
    // halo: each sweep invalidates 2 (five-point) or 4 (nine-point) columns at
    // each edge of the strip, the residual and the restriction one more each
    const TileGeo g = level_tiles(h, l, nine ? 4 * nu + 2 : 2 * nu + 2);
    T *out = ualt<T>(h, l);
    const dim3 grid = tile_grid(g), blk(FW);
#define PRE(NINE, NU) hipLaunchKernelGGL((k_pre<T, NINE, NU>), grid, blk, 0, h->st, F, out, C, Cl, g, stop)
#define PREW(NINE, NU) hipLaunchKernelGGL((k_pre<T, NINE, NU, true>), grid, blk, 0, h->st, F, out, C, Cl, g, stop)
#define PRE4(NU) hipLaunchKernelGGL((k_pre4<T, NU>), grid, blk, 0, h->st, F, out, C, Cl, g, stop)
    // Five-point FP64 levels with operator-induced weights compute them in the
    // pass instead of reading the 8 planes (16 of 68 bytes per fine point).
    // Not FP32 levels (their weights are the rounded FP64 ones), not learned
    // weights (no formula), and not nine-point levels, whose divisions cost
    // more time than the loads they replace.
    const bool wrec = pre_weights_in_pass<T>(h, l, nine);
    // small nine-point levels: every sweep inside one square tile's LDS copy
    const bool sq = square_tiles(h, l) && nu <= 2;
    // stencil once and b, u read, u written for each right-hand side on the
    // fine level; b and u (zero) written for each on the coarse level, and the
    // 8 weight planes read once unless computed
    const double K = h->nrhs;
    trace_begin(h, BMG_TRACE_PRE, l,
                sizeof(T) * ((stencil_planes(nine) + 3.0 * K) * (double)F.n * F.n +
                             (2.0 * K + (wrec ? 0.0 : 8.0)) * (double)Cl.n * Cl.n));
    if (sq) {
        const dim3 g2((F.n + T2D - 1) / T2D, (F.n + T2D - 1) / T2D);
        if (nu == 1)
            hipLaunchKernelGGL((k_pre2d<T, 1>), g2, dim3(T2D_THREADS), 0, h->st, F, out, C, Cl, stop);
        else
            hipLaunchKernelGGL((k_pre2d<T, 2>), g2, dim3(T2D_THREADS), 0, h->st, F, out, C, Cl, stop);
    } else if (wrec) {
        if constexpr (std::is_same<T, double>::value) {
            if (nu == 1) PREW(false, 1); else if (nu == 2) PREW(false, 2); else PREW(false, 3);
        }
    } else if (nine) {
        if (nu == 1) PRE(true, 1); else if (nu == 2) PRE(true, 2); else PRE(true, 3);
    } else if (BMG_FIVE_POINT_STEP_ROWS == 4) {
        if (nu == 1) PRE4(1); else if (nu == 2) PRE4(2); else PRE4(3);
    } else {
        if (nu == 1) PRE(false, 1); else if (nu == 2) PRE(false, 2); else PRE(false, 3);
    }
    trace_end(h, BMG_TRACE_PRE, l);
#undef PRE
#undef PREW
#undef PRE4
    LAUNCHCHK();
    std::swap(F.u, ualt<T>(h, l));
    return BMG_OK;
}

// Interpolation and nu sweeps in one pass; with `norm` (FP64 fine level) the
// tiles also leave partial sums of the squared accurate residual in h->part
// (their count in h->norm_parts; 0 if the pass could not fuse it).
template <typename T>
bmg_status fused_post(bmg_solver *h, int l, int nu, const int *stop, bool norm = false)
{
    Lev<T> &F = levm<T>(h, l);
    const Lev<T> &Cl = lev<T>(h, l + 1);
    const Wts<T> &C = wts<T>(h, l);
    const bool nine = h->nine[l];
    h->norm_parts = 0;
    if (nu < 1 || nu > 2) {
        TRY(interp<T>(h, F, C, Cl, stop));
        return smooth<T>(h, F, nine, nu, stop, l);
    }
    // halo: the edge lanes are never interpolated (stale from the start), then
    // each sweep invalidates 2 (five-point) or 4 (nine-point) more columns and
    // the fused residual one more
    const TileGeo g = level_tiles(h, l, nine ? 4 * nu + 2 : 2 * nu + 2);
    // small nine-point levels without the norm: every sweep inside one square
    // tile's LDS copy
    const bool sq = !norm && square_tiles(h, l);
    norm = norm && std::is_same<T, double>::value && g.ntiles <= NPART;
    T *out = ualt<T>(h, l);
    const dim3 grid = tile_grid(g), blk(FW);
#define POST(NINE, NU, NORM) \
    hipLaunchKernelGGL((k_post<T, NINE, NU, NORM>), grid, blk, 0, h->st, F, out, C, (const T *)Cl.u, g, h->part, stop)
#define POST4(NU, NORM) \
    hipLaunchKernelGGL((k_post4<T, NU, NORM>), grid, blk, 0, h->st, F, out, C, (const T *)Cl.u, g, h->part, stop)
    // stencil once and b, u read, u written for each right-hand side on the
    // fine level; the coarse correction of each and the 8 weight planes read
    const double K = h->nrhs;
    trace_begin(h, BMG_TRACE_POST, l,
                sizeof(T) * ((stencil_planes(nine) + 3.0 * K) * (double)F.n * F.n + (K + 8.0) * (double)Cl.n * Cl.n));
    if (sq) {
        const dim3 g2((F.n + T2D - 1) / T2D, (F.n + T2D - 1) / T2D);
        if (nu == 1)
            hipLaunchKernelGGL((k_post2d<T, 1>), g2, dim3(T2D_THREADS), 0, h->st, F, out, C, (const T *)Cl.u, stop);
        else
            hipLaunchKernelGGL((k_post2d<T, 2>), g2, dim3(T2D_THREADS), 0, h->st, F, out, C, (const T *)Cl.u, stop);
    } else if (!nine && BMG_FIVE_POINT_STEP_ROWS == 4) {
        if (norm) { if (nu == 1) POST4(1, true); else POST4(2, true); }
        else { if (nu == 1) POST4(1, false); else POST4(2, false); }
    } else if (norm) {
        if (nine) { if (nu == 1) POST(true, 1, true); else POST(true, 2, true); }
        else { if (nu == 1) POST(false, 1, true); else POST(false, 2, true); }
    } else {
        if (nine) { if (nu == 1) POST(true, 1, false); else POST(true, 2, false); }
        else { if (nu == 1) POST(false, 1, false); else POST(false, 2, false); }
    }
    trace_end(h, BMG_TRACE_POST, l);
#undef POST
#undef POST4
    LAUNCHCHK();
    std::swap(F.u, ualt<T>(h, l));
    if (norm) h->norm_parts = g.ntiles;
    return BMG_OK;
}

// Coarse levels of at most persistent_below_n points per side: their whole
// sub-cycle in one workgroup (k_small_vcycle), iterates and right-hand sides in
// LDS.

template <typename T>
bmg_status small_cycle(bmg_solver *h, int l, const int *stop)
{
    SmallH<T> S{};
    S.nl = h->nlev - l;
    if (S.nl > SMALL_MAXL) return fail(BMG_EINVAL, "too many small levels");
    if (lev<T>(h, l).n > SMALL_MAX_N) return fail(BMG_EINVAL, "level %d too large for one workgroup", l);
    for (int k = 0; k < S.nl; ++k) {
        S.L[k] = lev<T>(h, l + k);
        if (k + 1 < S.nl) S.C[k] = wts<T>(h, l + k);
    }
    const int off = small_layout(S);
    S.band = h->band;
    S.nu1 = h->opt.nu1;
    S.nu2 = h->opt.nu2;
    S.ks0 = h->ks[l];
    S.kstop = h->kstop;
    const size_t shmem = (size_t)off * sizeof(T);
    if (shmem > SMALL_LDS_MAX)
        return fail(BMG_EINVAL, "levels %d..%d need %zu bytes of LDS in one workgroup (at most %d)", l,
                    h->nlev - 1, shmem, SMALL_LDS_MAX);
    static bool attr_set[2] = {false, false};
    const int which = sizeof(T) == 8 ? 0 : 1;
    if (!attr_set[which]) {
        HIPCHK(hipFuncSetAttribute((const void *)k_small_vcycle<T, true>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, SMALL_LDS_MAX));
        attr_set[which] = true;
    }
    hipLaunchKernelGGL((k_small_vcycle<T, true>), dim3(h->nrhs), dim3(SMALL_THREADS), shmem, h->st, S, stop);
    LAUNCHCHK();
    return BMG_OK;
}

template <typename T>
bmg_status fused_cycle_from(bmg_solver *h, int l, const int *stop, bool norm)
{
    if (l == h->nlev - 1) return coarse<T>(h, lev<T>(h, l), stop);
    if (l >= 1 && lev<T>(h, l).n <= persistent_of(h->opt)) return small_cycle<T>(h, l, stop);
    TRY(fused_pre<T>(h, l, h->opt.nu1, stop));
    TRY(fused_cycle_from<T>(h, l + 1, stop, false));
    return fused_post<T>(h, l, h->opt.nu2, stop, norm && l == 0);
}

bmg_status fused_vcycle(bmg_solver *h, const int *stop, bool norm = false)
{
    return fused_cycle_from<double>(h, 0, stop, norm);
}
bmg_status fused_vcycle32(bmg_solver *h, const int *stop) { return fused_cycle_from<float>(h, 0, stop, false); }

// A refinement step's cycle with the fine post pass adding the correction to
// (XH, XL) itself (k_post_ir): a five-point fine level, a post sweep count the
// pass takes, one right-hand side.  With an FP32 inner cycle the fine pre pass
// also takes the scaled residual itself (k_pre_ir).
static bool post_update_fusable(const bmg_solver *h)
{
    return h->opt.kernels == BMG_KERNELS_FUSED && h->opt.smoother == BMG_SMOOTH_POINT && !h->nine[0] &&
           BMG_FIVE_POINT_STEP_ROWS == 2 && h->nrhs == 1 && h->nlev >= 2 && h->opt.nu2 >= 1 && h->opt.nu2 <= 2;
}

static bool ir_fusable(const bmg_solver *h)
{
    return post_update_fusable(h) && h->opt.nu1 >= 1 && h->opt.nu1 <= 3 && h->L32[0].ld == h->L[0].ld;
}

// The fine post pass of such a step: interpolation and sweeps, then
// (XH, XL) += s u at every owned point.
template <typename T>
static bmg_status post_update(bmg_solver *h, const int *stop, const IrArgs &ir)
{
    const Lev<T> &F = lev<T>(h, 0);
    const Lev<T> &Cl = lev<T>(h, 1);
    const Wts<T> &C = wts<T>(h, 0);
    const int nu2 = h->opt.nu2;
    const double nf = (double)F.n * F.n, ncc = (double)Cl.n * Cl.n;
    const TileGeo g = level_tiles(h, 0, 2 * nu2 + 2);
    const dim3 grid = tile_grid(g), blk(FW);
    // stencil, b and u read, (XH, XL) read and written; the coarse correction
    // and the 8 weight planes read
    trace_begin(h, BMG_TRACE_POST, 0, sizeof(T) * ((stencil_planes(false) + 2.0) * nf + 9.0 * ncc) + 32.0 * nf);
    if (nu2 == 1)
        hipLaunchKernelGGL((k_post_ir<T, 1>), grid, blk, 0, h->st, F, C, (const T *)Cl.u, g, stop, ir);
    else
        hipLaunchKernelGGL((k_post_ir<T, 2>), grid, blk, 0, h->st, F, C, (const T *)Cl.u, g, stop, ir);
    trace_end(h, BMG_TRACE_POST, 0);
    LAUNCHCHK();
    return BMG_OK;
}

static bmg_status ir_fused_cycle(bmg_solver *h, const int *stop, const IrArgs &ir)
{
    Lev<float> &F = h->L32[0];
    const Lev<float> &Cl = h->L32[1];
    const Wts<float> &C = h->C32[0];
    const int nu1 = h->opt.nu1;
    const double nf = (double)F.n * F.n, ncc = (double)Cl.n * Cl.n;
    const TileGeo g = level_tiles(h, 0, 2 * nu1 + 2);
    const dim3 grid = tile_grid(g), blk(FW);
    // stencil and the FP64 residual read, u and b written; b and u (zero)
    // written on the coarse level and the 8 weight planes read
    trace_begin(h, BMG_TRACE_PRE, 0, 4.0 * ((stencil_planes(false) + 2.0) * nf + 10.0 * ncc) + 8.0 * nf);
#define PREI(NU) hipLaunchKernelGGL((k_pre_ir<NU>), grid, blk, 0, h->st, F, h->ualt32[0], C, Cl, g, stop, ir)
    if (nu1 == 1) PREI(1); else if (nu1 == 2) PREI(2); else PREI(3);
#undef PREI
    trace_end(h, BMG_TRACE_PRE, 0);
    LAUNCHCHK();
    std::swap(F.u, h->ualt32[0]);
    TRY(fused_cycle_from<float>(h, 1, stop, false));
    return post_update<float>(h, stop, ir);
}

// Sum of squares of r = b - A u (res) or of the array x, into scal[slot]; with
// record, also the history / stop bookkeeping of the running solve.
template <typename T>
bmg_status sumsq(bmg_solver *h, const Lev<T> &L, bool nine, bool res, const T *x, int slot,
                 bool record, double tol, int maxc)
{
    const int nb = std::min(NPART_ROWS, L.n);
    const int *stop = record ? h->stop : nullptr;
    trace_begin(h, BMG_TRACE_RESNORM, 0,
                sizeof(T) * (res ? stencil_planes(nine) + 2.0 : 1.0) * (double)L.n * L.n);
    if (res) {
        if (nine) hipLaunchKernelGGL((k_sumsq_partial<T, true, true>), dim3(nb), dim3(256), 0, h->st, L, x, h->part, stop);
        else hipLaunchKernelGGL((k_sumsq_partial<T, false, true>), dim3(nb), dim3(256), 0, h->st, L, x, h->part, stop);
    } else {
        hipLaunchKernelGGL((k_sumsq_partial<T, false, false>), dim3(nb), dim3(256), 0, h->st, L, x, h->part, stop);
    }
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(1024), 0, h->st, (const double *)h->part, nb,
                       h->scal + slot, record ? h->hist : nullptr, h->count, h->stop,
                       (const double *)(h->scal + S_BNORM), tol, maxc, 0.0);
    trace_end(h, BMG_TRACE_RESNORM, 0);
    LAUNCHCHK();
    return BMG_OK;
}

// Accurate residual of (XH, XL) against B on the fine level, its sum of
// squares into scal[slot] and, with record, the history / stop bookkeeping
// (refine > 0: raise the switch-to-refinement code at that residual).
// mode: 0 norm only, 1 r -> rout, 2 r -> L0.b and 0 -> L0.u.
bmg_status resnorm_dd(bmg_solver *h, const double *B, const double *XH, const double *XL, int mode,
                      double *rout, int slot, bool record, double tol, int maxc, double refine)
{
    const Lev<double> &L = h->L[0];
    const int nb = std::min(NPART_ROWS, L.n);
    const int *stop = record ? h->stop : nullptr;
    const dim3 g(nb), b(256);
#define RDD(NINE, MODE) hipLaunchKernelGGL((k_resid_dd<NINE, MODE>), g, b, 0, h->st, L, B, XH, XL, rout, h->part, stop)
    // stencil, B and XH (and XL) read; r (mode 1) or b and u (mode 2) written
    trace_begin(h, BMG_TRACE_RESNORM, 0,
                8.0 * (stencil_planes(h->nine[0]) + (XL ? 3.0 : 2.0) + (mode == 1 ? 1.0 : mode == 2 ? 2.0 : 0.0)) *
                    (double)L.n * L.n);
    if (h->nine[0]) {
        if (mode == 0) RDD(true, 0); else if (mode == 1) RDD(true, 1); else RDD(true, 2);
    } else {
        if (mode == 0) RDD(false, 0); else if (mode == 1) RDD(false, 1); else RDD(false, 2);
    }
#undef RDD
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(1024), 0, h->st, (const double *)h->part, nb,
                       h->scal + slot, record ? h->hist : nullptr, h->count, h->stop,
                       (const double *)(h->scal + S_BNORM), tol, maxc, refine);
    trace_end(h, BMG_TRACE_RESNORM, 0);
    LAUNCHCHK();
    return BMG_OK;
}

bmg_status read_scalars(bmg_solver *h, double *dst, int first, int count)
{
    HIPCHK(hipMemcpyAsync(dst, h->scal + first, count * sizeof(double), hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return BMG_OK;
}

bmg_status pack_in(bmg_solver *h, const double *src, double *dst)
{
    const Lev<double> &L = h->L[0];
    hipLaunchKernelGGL((k_pack_in<double, double>), grid2(L.n, L.n, B2), B2, 0, h->st, src, L.n, dst, L.ld);
    LAUNCHCHK();
    return BMG_OK;
}

bmg_status pack_out(bmg_solver *h, const double *src, double *dst)
{
    const Lev<double> &L = h->L[0];
    hipLaunchKernelGGL((k_pack_out<double, double>), grid2(L.n, L.n, B2), B2, 0, h->st, src, L.ld, L.n, dst);
    LAUNCHCHK();
    return BMG_OK;
}

// eps * || |A| |XH| + |B| || into scal[S_FLOOR] (unnormalised).
bmg_status floor_sum(bmg_solver *h, const double *B, const double *XH)
{
    const Lev<double> &L = h->L[0];
    const int nb = std::min(NPART_ROWS, L.n);
    if (h->nine[0]) hipLaunchKernelGGL((k_floor_partial<true>), dim3(nb), dim3(256), 0, h->st, L, B, XH, h->part);
    else hipLaunchKernelGGL((k_floor_partial<false>), dim3(nb), dim3(256), 0, h->st, L, B, XH, h->part);
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(1024), 0, h->st, (const double *)h->part, nb, h->scal + S_FLOOR,
                       nullptr, h->count, h->stop, (const double *)(h->scal + S_BNORM), 0.0, 0, 0.0);
    LAUNCHCHK();
    return BMG_OK;
}

}  // namespace

namespace bmgi {

bmg_status solve_level(bmg_solver *h, int l, double tol, int maxc, int *cycles)
{
    const Lev<double> &L = h->L[l];
    *cycles = 0;
    HIPCHK(hipMemsetAsync(L.u, 0, (size_t)(L.n + 2) * L.ld * sizeof(double), h->st));
    TRY(sumsq<double>(h, L, false, false, L.b, S_TMP, false, 0.0, 0));
    double v[S_NSCAL];
    TRY(read_scalars(h, v, 0, 4));
    if (v[S_TMP] == 0.0) return BMG_OK;
    const double nb = sqrt(v[S_TMP]);
    const int np = std::min(NPART_ROWS, L.n);
    for (int k = 0; k < maxc; ++k) {
        TRY(vcycle_from<double>(h, l, nullptr));
        if (h->nine[l])
            hipLaunchKernelGGL((k_resid_dd<true, 0>), dim3(np), dim3(256), 0, h->st, L, (const double *)L.b,
                               (const double *)L.u, nullptr, nullptr, h->part, nullptr);
        else
            hipLaunchKernelGGL((k_resid_dd<false, 0>), dim3(np), dim3(256), 0, h->st, L, (const double *)L.b,
                               (const double *)L.u, nullptr, nullptr, h->part, nullptr);
        hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(1024), 0, h->st, (const double *)h->part, np,
                           h->scal + S_SUMSQ, nullptr, h->count, h->stop, (const double *)(h->scal + S_BNORM), 0.0,
                           0, 0.0);
        LAUNCHCHK();
        TRY(read_scalars(h, v, 0, 4));
        *cycles = k + 1;
        if (!(sqrt(v[S_SUMSQ]) / nb > tol)) break;
    }
    return BMG_OK;
}

}  // namespace bmgi

// ================================================================ C API
extern "C" {

const char *bmg_last_error(void) { return g_err; }

const char *bmg_status_string(int s)
{
    switch (s) {
    case BMG_OK: return "ok";
    case BMG_EINVAL: return "invalid argument";
    case BMG_EBREAKDOWN: return "breakdown (non-positive interpolation denominator or coarse pivot)";
    case BMG_ENOCONV: return "not converged within max_cycles";
    case BMG_EDIVERGED: return "diverged";
    case BMG_EDEVICE: return "HIP runtime error";
    case BMG_EWORKSPACE: return "workspace missing, too small or misaligned";
    default: return "unknown status";
    }
}

bmg_status bmg_default_options(bmg_options *o)
{
    if (!o) return fail(BMG_EINVAL, "options pointer is NULL");
    memset(o, 0, sizeof *o);
    o->nu1 = 2;
    o->nu2 = 1;
    o->max_cycles = 100;
    o->precision = BMG_FP64;
    o->kernels = BMG_KERNELS_FUSED;
    o->check_every = 8;
    o->refine_factor = 16;
    return BMG_OK;
}

bmg_status bmg_workspace_bytes(int n, int kind, const bmg_options *o, size_t *bytes)
{
    if (!bytes) return fail(BMG_EINVAL, "bytes pointer is NULL");
    if (!valid_n(n)) return fail(BMG_EINVAL, "n=%d is not 2^m-1 with 2 <= m <= 15", n);
    if (kind != 5 && kind != 9) return fail(BMG_EINVAL, "stencil kind %d is not 5 or 9", kind);
    bmg_options d;
    bmg_default_options(&d);
    const bmg_options &op = o ? *o : d;
    TRY(check_options(op));
    if (coarsest_of(op) > n) return fail(BMG_EINVAL, "coarsest_n=%d exceeds n=%d", op.coarsest_n, n);
    *bytes = plan(nullptr, n, kind, op, nullptr);
    return BMG_OK;
}

bmg_status bmg_discretize(const double *k, const double *f, int n, double *stencil, double *rhs,
                          bmg_stream stream)
{
    if (!valid_n(n)) return fail(BMG_EINVAL, "n=%d is not 2^m-1 with 2 <= m <= 15", n);
    if (!k || !f || !stencil || !rhs) return fail(BMG_EINVAL, "NULL array");
    int m = 0;
    while ((1 << m) < n + 1) ++m;
    const double h2 = ldexp(1.0, -2 * m);
    hipLaunchKernelGGL(k_discretize, grid2(n, n, B2), B2, 0, (hipStream_t)stream, k, f, n, h2, stencil, rhs);
    LAUNCHCHK();
    return BMG_OK;
}

}  // extern "C"

// The set-up of bmg_setup into the handle h (fresh), after the arguments have
// been checked; on failure the caller releases h.
static bmg_status setup_into(bmg_solver *h, const double *stencil, int n, int kind, const bmg_options &op,
                             void *workspace, size_t ws_bytes, size_t need, bmg_stream stream)
{
    h->n = n;
    h->kind = kind;
    h->opt = op;
    h->st = (hipStream_t)stream;
    h->ws = (char *)workspace;
    h->ws_bytes = ws_bytes;
    plan(h, n, kind, op, h->ws);
    auto bail = [&](bmg_status s) { return s; };
#define SCHK(x)                                  \
    do {                                         \
        bmg_status s_ = (x);                     \
        if (s_ != BMG_OK) return bail(s_);       \
    } while (0)
    if (hipMemsetAsync(h->ws, 0, need, h->st) != hipSuccess)
        return bail(fail(BMG_EDEVICE, "hipMemsetAsync of the workspace failed"));
    hipLaunchKernelGGL(k_import_stencil, grid2(n, n, B2), B2, 0, h->st, stencil, kind, h->L[0], h->flags);
    auto boxmg_weights = [&](int l) {
        const int nc = h->L[l + 1].n;
        launch_weights(h->L[l], h->C[l], nc, h->flags, grid2(nc + 1, nc + 1, B2), B2, h->st);
    };
    auto galerkin = [&](int l) {
        launch_rap(h->L[l], h->C[l], h->L[l + 1], h->st);
    };
    // levels whose weights come from the network: the first `cut`.  A coarse
    // operator built with the network's weights can leave BoxMG's formula a
    // denominator <= 0 on a level below (the network corrects weights, it
    // does not keep the coarse operators M-matrices).  The last level above it
    // that used the network then takes BoxMG's weights, and it and every level
    // below are formed again; this repeats while learned levels are left.  A
    // breakdown with no learned level above it (the fine level's own operator)
    // stays an error.
    int cut = 0;
    if (op.interp == BMG_INTERP_LEARNED)
        cut = op.learned_levels == 0 ? h->nlev - 1 : std::min(op.learned_levels, h->nlev - 1);
    for (int l = 0; l + 1 < h->nlev;) {
        if (l < cut) SCHK(net_level_weights(op.net, h->L[l], h->nine[l], h->C[l], h->flags, h->st));
        else boxmg_weights(l);
        if (l >= 1 && cut > 0) {
            int fl = 0;
            if (hipMemcpyAsync(&fl, h->flags, sizeof fl, hipMemcpyDeviceToHost, h->st) != hipSuccess ||
                hipStreamSynchronize(h->st) != hipSuccess)
                return bail(fail(BMG_EDEVICE, "reading the set-up flags failed"));
            if (fl & F_BREAK_INTERP) {
                const int cleared = fl & ~F_BREAK_INTERP;
                if (hipMemcpyAsync(h->flags, &cleared, sizeof cleared, hipMemcpyHostToDevice, h->st) != hipSuccess ||
                    hipStreamSynchronize(h->st) != hipSuccess)
                    return bail(fail(BMG_EDEVICE, "writing the set-up flags failed"));
                cut = std::min(cut, l) - 1;
                l = cut;
                continue;
            }
        }
        galerkin(l);
        ++l;
    }
    h->learned_used = cut;
    hipLaunchKernelGGL(k_band_factor, dim3(1), dim3(BAND_FACTOR_THREADS), 0, h->st, h->L[h->nlev - 1], h->Lb, h->Dd,
                       h->flags);
    hipLaunchKernelGGL(k_band_expand, dim3(h->band.M / 4), dim3(256), 0, h->st, h->band.nc, (const double *)h->Lb,
                       (const double *)h->Dd, (double *)h->band.CF, (double *)h->band.CG, (double *)h->band.Dp);
    if (op.smoother == BMG_SMOOTH_LINE) {
        // y-lines in the grid's frame; x-lines on the transposed O (in the
        // scratch plane) and W
        for (int l = 0; l < h->nlev; ++l) {
            const Lev<double> &L = h->L[l];
            const dim3 fb(64), fg((L.n + 63) / 64), tb(LT, 8), tg((L.n + 2 + LT - 1) / LT, (L.n + 2 + LT - 1) / LT);
            hipLaunchKernelGGL(k_line_factor, fg, fb, 0, h->st, L.n, L.ld, (const double *)L.O, (const double *)L.S,
                               h->lfy[l], h->rfy[l], h->flags);
            hipLaunchKernelGGL(k_transpose, tg, tb, 0, h->st, L.n, L.ld, (const double *)L.O, h->lineD);
            hipLaunchKernelGGL(k_transpose, tg, tb, 0, h->st, L.n, L.ld, (const double *)L.W, h->WT[l]);
            hipLaunchKernelGGL(k_line_factor, fg, fb, 0, h->st, L.n, L.ld, (const double *)h->lineD,
                               (const double *)h->WT[l], h->lfx[l], h->rfx[l], h->flags);
        }
    }
    if (h->f32) {
        // the FP32 hierarchy: every plane and weight array rounded, in one
        // launch per list of arrays (the small levels would otherwise be
        // dozens of launches of a few microseconds each)
        RoundList R{};
        size_t most = 0;
        auto flush = [&]() {
            if (R.n == 0) return;
            const dim3 g((unsigned)std::min<size_t>((most + 255) / 256, 1024), (unsigned)R.n), b(256);
            hipLaunchKernelGGL(k_round_f32_list, g, b, 0, h->st, R);
            R.n = 0;
            most = 0;
        };
        auto add = [&](const double *src, float *dst, size_t count) {
            if (R.n == ROUND_MAX) flush();
            R.src[R.n] = src;
            R.dst[R.n] = dst;
            R.count[R.n] = count;
            ++R.n;
            most = std::max(most, count);
        };
        for (int l = 0; l < h->nlev; ++l) {
            const size_t pl = (size_t)(h->L[l].n + 2) * h->L[l].ld;
            add(h->L[l].O, h->L32[l].O, pl);
            add(h->L[l].W, h->L32[l].W, pl);
            add(h->L[l].S, h->L32[l].S, pl);
            if (h->nine[l]) {
                add(h->L[l].SW, h->L32[l].SW, pl);
                add(h->L[l].NW, h->L32[l].NW, pl);
            }
            if (l + 1 < h->nlev) add(h->C[l].p, h->C32[l].p, 8 * h->C[l].ps);
        }
        flush();
    }
    if (hipGetLastError() != hipSuccess) return bail(fail(BMG_EDEVICE, "set-up kernel launch failed"));
    int flags = 0;
    if (hipMemcpyAsync(&flags, h->flags, sizeof flags, hipMemcpyDeviceToHost, h->st) != hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess)
        return bail(fail(BMG_EDEVICE, "reading the set-up flags failed"));
    if (flags & (F_NONFINITE | F_DIAG | F_BOUNDARY | F_ASYM))
        return bail(fail(BMG_EINVAL, "stencil rejected:%s%s%s%s", (flags & F_NONFINITE) ? " non-finite entry" : "",
                         (flags & F_DIAG) ? " centre <= 0" : "", (flags & F_BOUNDARY) ? " coupling to the boundary" : "",
                         (flags & F_ASYM) ? " not symmetric" : ""));
    if (flags & (F_BREAK_INTERP | F_BREAK_COARSE | F_BREAK_LINE))
        return bail(fail(BMG_EBREAKDOWN, "%s", (flags & F_BREAK_INTERP)   ? "interpolation denominator <= 0"
                                               : (flags & F_BREAK_COARSE) ? "coarsest pivot <= 0"
                                                                          : "line factor pivot <= 0"));
#undef SCHK
    return BMG_OK;
}

// Arguments of bmg_setup, checked; *need receives the workspace bytes.
static bmg_status check_setup(const double *stencil, int n, int kind, const bmg_options *o, bmg_options *op,
                              size_t *need)
{
    if (!valid_n(n)) return fail(BMG_EINVAL, "n=%d is not 2^m-1 with 2 <= m <= 15", n);
    if (kind != 5 && kind != 9) return fail(BMG_EINVAL, "stencil kind %d is not 5 or 9", kind);
    if (!stencil) return fail(BMG_EINVAL, "stencil is NULL");
    bmg_default_options(op);
    if (o) *op = *o;
    TRY(check_options(*op));
    if (coarsest_of(*op) > n) return fail(BMG_EINVAL, "coarsest_n=%d exceeds n=%d", op->coarsest_n, n);
    *need = plan(nullptr, n, kind, *op, nullptr);
    return BMG_OK;
}

extern "C" {

bmg_status bmg_setup(bmg_solver **out, const double *stencil, int n, int kind, const bmg_options *o,
                     void *workspace, size_t ws_bytes, bmg_stream stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!out) return fail(BMG_EINVAL, "out pointer is NULL");
    *out = nullptr;
    bmg_options op;
    size_t need = 0;
    TRY(check_setup(stencil, n, kind, o, &op, &need));
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace & (ALIGN - 1)))
        return fail(BMG_EWORKSPACE, "workspace %p of %zu bytes; need %zu bytes, 256-byte aligned",
                    workspace, ws_bytes, need);
    bmg_solver *h = new bmg_solver();
    const bmg_status s = setup_into(h, stencil, n, kind, op, workspace, ws_bytes, need, stream);
    if (s != BMG_OK) {
        delete h;
        return s;
    }
    h->t_setup_ms = ms_since(t0);
    *out = h;
    return BMG_OK;
}

bmg_status bmg_destroy(bmg_solver *h)
{
    if (!h) return BMG_OK;
    for (hipEvent_t e : h->tr_ev) (void)hipEventDestroy(e);
    if (h->pair_exec) (void)hipGraphExecDestroy(h->pair_exec);
    if (h->cap_st) (void)hipStreamDestroy(h->cap_st);
    delete h;
    return BMG_OK;
}

// The fused passes relax pointwise: line relaxation runs the unfused cycle.
static bool fused(const bmg_solver *h)
{
    return h->opt.kernels == BMG_KERNELS_FUSED && h->opt.smoother == BMG_SMOOTH_POINT;
}

// One FP64 V-cycle on the level-0 arrays (b, u already set).
static bmg_status cycle64(bmg_solver *h, const int *stop)
{
    if (fused(h)) return fused_vcycle(h, stop);
    return vcycle_from<double>(h, 0, stop);
}

// One FP32 refinement step: r = B0 - A (XH + XL) is in L0.r and the residual
// pass left the partial maxima of |r| after its partial sums; scale to the
// power of two s >= ||r||_inf, round to FP32, V32 from zero, (XH, XL) += s d32.
// The scaling and the update run inside the fine level's passes where the
// cycle allows (the same values), else as passes of their own.
static bmg_status ir_correct(bmg_solver *h, const int *stop)
{
    const Lev<double> &L = h->L[0];
    const Lev<float> &F = h->L32[0];
    const int nb = std::min(NPART_ROWS, L.n);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(1024), 0, h->st, (const double *)h->part + nb, nb,
                       h->scal + S_RMAX, stop);
    if (ir_fusable(h)) {
        LAUNCHCHK();
        const IrArgs ir{L.r, h->scal + S_RMAX, h->scal + S_SCALE, h->XH, h->XL};
        return ir_fused_cycle(h, stop, ir);
    }
    hipLaunchKernelGGL(k_ir_scale, grid2(L.n, L.n, B2), B2, 0, h->st, L, F, (const double *)(h->scal + S_RMAX),
                       h->scal + S_SCALE, stop);
    LAUNCHCHK();
    if (fused(h)) TRY(fused_vcycle32(h, stop));
    else TRY(vcycle_from<float>(h, 0, stop));
    hipLaunchKernelGGL(k_dd_update, grid2(L.n, L.n, B2), B2, 0, h->st, L, h->XH, h->XL, (const float *)F.u,
                       (const double *)(h->scal + S_SCALE), stop);
    LAUNCHCHK();
    return BMG_OK;
}

// One plain FP64 cycle of the solve and its recorded accurate residual norm:
// fused into the fine level's last pass when the fused path can, else a
// separate residual pass.
static bmg_status cycle_and_norm(bmg_solver *h, double tol, int maxc, double refine)
{
    const Lev<double> &L = h->L[0];
    if (fused(h)) {
        TRY(fused_vcycle(h, h->stop, true));
        if (h->norm_parts > 0) {
            trace_begin(h, BMG_TRACE_RESNORM, 0, 8.0 * h->norm_parts);   // the partial sums
            hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(1024), 0, h->st, (const double *)h->part,
                               h->norm_parts, h->scal + S_SUMSQ, h->hist, h->count, h->stop,
                               (const double *)(h->scal + S_BNORM), tol, maxc, refine);
            trace_end(h, BMG_TRACE_RESNORM, 0);
            LAUNCHCHK();
            return BMG_OK;
        }
    } else {
        TRY(vcycle_from<double>(h, 0, h->stop));
    }
    return resnorm_dd(h, L.b, L.u, nullptr, 0, nullptr, S_SUMSQ, true, tol, maxc, refine);
}

// Rows per tile of k_postpre: two of its 72 KiB workgroups share a CU, so
// the fewest warm-up rows with all tiles in one round of 512 (148 rows at
// 4095^2: 18 strips x 28 tiles).
static int postpre_tile_rows(const bmg_solver *h, int n, int hx)
{
    if (h->opt.tile_rows > 0) return h->opt.tile_rows;
    const int useful = FW - 2 * hx;
    const int strips = (n + useful - 1) / useful;
    const int rows = std::max(1, 512 / strips);
    return ((n + rows - 1) / rows + 1) & ~1;
}

// Tiles of k_postpre on the fine level: halo for the interpolation edge, the
// sweeps, the residual and the restriction.
static TileGeo postpre_geo(const bmg_solver *h)
{
    const int hx = 2 * (h->opt.nu1 + 1) + 4;
    return tile_geo(h->L[0].n, hx, postpre_tile_rows(h, h->L[0].n, hx));
}

// Plain FP64 cycles where the fine post pass of each cycle runs together with
// the fine pre pass of the next (k_postpre): an FP64 five-point fine level
// with one right-hand side (operator-induced or learned weights: the pass
// reads the stored ones), one post sweep and one or two pre sweeps, and at
// most NPART tiles (their norm partials).
static bool postpre_ok(const bmg_solver *h)
{
    return !h->f32 && h->opt.kernels == BMG_KERNELS_FUSED && h->opt.smoother == BMG_SMOOTH_POINT && !h->nine[0] &&
           BMG_FIVE_POINT_STEP_ROWS == 2 && h->nlev >= 2 && h->opt.nu2 == 1 && (h->opt.nu1 == 1 || h->opt.nu1 == 2) &&
           h->nrhs == 1 && postpre_geo(h).ntiles <= NPART;
}

// One plain FP64 cycle and its recorded norm on the k_postpre schedule.
// *pending: the fine pre pass of this cycle already ran inside the last
// k_postpre, its iterate in L0.r (free on this schedule).  Level 0 rotates
// three buffers: the pass reads u' and writes u_k and the next u''; level 1
// takes u_c = 0 in its second buffer, since e_c is read until the pass ends.
static bmg_status cycle_and_norm_pp(bmg_solver *h, double tol, int maxc, double refine, bool *pending)
{
    Lev<double> &F = h->L[0];
    Lev<double> &C1 = h->L[1];
    const int nb = h->opt.nu1;
    if (!*pending) TRY(fused_pre<double>(h, 0, nb, h->stop));
    TRY(fused_cycle_from<double>(h, 1, h->stop, false));
    // u_k goes where L0.u points once a pre pass is pending, so that L0.u
    // keeps the last result when the stop flag makes later passes return
    double *in = *pending ? F.r : F.u;
    double *const bufs[3] = {F.u, h->ualt[0], F.r};
    double *out[2];
    int m = 0;
    for (double *b : bufs)
        if (b != in) out[m++] = b;
    Lev<double> Fin = F;
    Fin.u = in;
    const TileGeo g = postpre_geo(h);
    const dim3 grid = tile_grid(g), blk(FW);
    const double nf = (double)F.n * F.n, ncc = (double)C1.n * C1.n;
    // stencil, b and u' read, u_k and u'' written; e_c and the 8 weight planes
    // read, b_c and u_c written
    trace_begin(h, BMG_TRACE_POSTPRE, 0, 8.0 * ((stencil_planes(false) + 4.0) * nf + 11.0 * ncc));
    if (nb == 1)
        hipLaunchKernelGGL((k_postpre<1>), grid, blk, 0, h->st, Fin, out[0], out[1], h->C[0], (const double *)C1.u, C1,
                           h->ualt[1], g, h->part, h->stop);
    else
        hipLaunchKernelGGL((k_postpre<2>), grid, blk, 0, h->st, Fin, out[0], out[1], h->C[0], (const double *)C1.u, C1,
                           h->ualt[1], g, h->part, h->stop);
    trace_end(h, BMG_TRACE_POSTPRE, 0);
    LAUNCHCHK();
    F.u = out[0];
    F.r = out[1];
    h->ualt[0] = in;
    std::swap(C1.u, h->ualt[1]);
    *pending = true;
    trace_begin(h, BMG_TRACE_RESNORM, 0, 8.0 * g.ntiles);
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(1024), 0, h->st, (const double *)h->part, g.ntiles,
                       h->scal + S_SUMSQ, h->hist, h->count, h->stop, (const double *)(h->scal + S_BNORM), tol, maxc,
                       refine);
    trace_end(h, BMG_TRACE_RESNORM, 0);
    LAUNCHCHK();
    return BMG_OK;
}

// The host state a cycle depends on: every level's buffer pointers.
static std::vector<void *> cycle_state(const bmg_solver *h)
{
    std::vector<void *> v;
    for (int l = 0; l < h->nlev; ++l) {
        v.push_back(h->L[l].u);
        v.push_back(h->L[l].r);
        v.push_back(h->ualt[l]);
    }
    return v;
}

// Two plain cycles on the k_postpre schedule (a pre pass pending) as one
// graph launch.  On the k_postpre schedule the level buffers rotate with
// period two, so a graph captured from one state leaves the host state as it
// found it and can be replayed for every later pair; the capture itself runs
// the host code of the two cycles (their buffer swaps included), and the
// captured graph is launched once to do their work.  The graph is rebuilt
// when the state or the stop-test arguments differ from the capture's.  The
// capture records on a stream of the handle's own (no work runs while it
// records), and the graph is launched on the solve's stream, which may be
// the null stream.
static bmg_status cycle_pair_graph(bmg_solver *h, double tol, int maxc, double refine, bool *pending)
{
    const std::vector<void *> s0 = cycle_state(h);
    if (h->pair_exec && (s0 != h->pair_state || tol != h->pair_tol || maxc != h->pair_maxc || refine != h->pair_refine)) {
        HIPCHK(hipStreamSynchronize(h->st));
        (void)hipGraphExecDestroy(h->pair_exec);
        h->pair_exec = nullptr;
    }
    if (h->pair_exec) {
        HIPCHK(hipGraphLaunch(h->pair_exec, h->st));
        return BMG_OK;
    }
    if (!h->cap_st) HIPCHK(hipStreamCreateWithFlags(&h->cap_st, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(h->cap_st, hipStreamCaptureModeThreadLocal));
    hipStream_t run = h->st;
    h->st = h->cap_st;
    bmg_status s = cycle_and_norm_pp(h, tol, maxc, refine, pending);
    if (s == BMG_OK) s = cycle_and_norm_pp(h, tol, maxc, refine, pending);
    h->st = run;
    const hipError_t ce = hipStreamEndCapture(h->cap_st, &g);
    if (s != BMG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (ce != hipSuccess || !g) return fail(BMG_EDEVICE, "capturing two cycles failed: %s", hipGetErrorString(ce));
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(BMG_EDEVICE, "instantiating the cycle graph failed: %s", hipGetErrorString(ie));
    HIPCHK(hipGraphLaunch(ex, h->st));
    if (cycle_state(h) == s0) {
        h->pair_exec = ex;
        h->pair_state = s0;
        h->pair_tol = tol;
        h->pair_maxc = maxc;
        h->pair_refine = refine;
    } else {
        HIPCHK(hipStreamSynchronize(h->st));
        (void)hipGraphExecDestroy(ex);
        h->pair_off = true;
    }
    return BMG_OK;
}

// One FP64 refinement step: L0.b holds r, L0.u = 0; V-cycle, (XH, XL) += u
// (inside the fine post pass where the cycle allows).
static bmg_status refine_step64(bmg_solver *h, const int *stop)
{
    const Lev<double> &L = h->L[0];
    if (post_update_fusable(h)) {
        TRY(fused_pre<double>(h, 0, h->opt.nu1, stop));
        TRY(fused_cycle_from<double>(h, 1, stop, false));
        const IrArgs ir{nullptr, nullptr, nullptr, h->XH, h->XL};
        return post_update<double>(h, stop, ir);
    }
    TRY(cycle64(h, stop));
    hipLaunchKernelGGL(k_dd_update, grid2(L.n, L.n, B2), B2, 0, h->st, L, h->XH, h->XL, (const float *)nullptr,
                       (const double *)nullptr, stop);
    LAUNCHCHK();
    return BMG_OK;
}

bmg_status bmg_vcycle(bmg_solver *h, const double *rhs, double *x, double *rel_res)
{
    if (!h || !rhs || !x) return fail(BMG_EINVAL, "NULL argument");
    const Lev<double> &L = h->L[0];
    if (h->f32) {
        TRY(pack_in(h, rhs, h->B0));
        TRY(pack_in(h, x, h->XH));
        HIPCHK(hipMemsetAsync(h->XL, 0, (size_t)(L.n + 2) * L.ld * sizeof(double), h->st));
        TRY(resnorm_dd(h, h->B0, h->XH, nullptr, 1, L.r, S_TMP, false, 0.0, 0, 0.0));
        TRY(ir_correct(h, nullptr));
        TRY(pack_out(h, h->XH, x));
        if (rel_res) {
            TRY(sumsq<double>(h, L, false, false, h->B0, S_TMP, false, 0.0, 0));
            TRY(resnorm_dd(h, h->B0, h->XH, h->XL, 0, nullptr, S_SUMSQ, false, 0.0, 0, 0.0));
        }
    } else {
        TRY(pack_in(h, rhs, L.b));
        TRY(pack_in(h, x, L.u));
        TRY(cycle64(h, nullptr));
        TRY(pack_out(h, L.u, x));
        if (rel_res) {
            TRY(sumsq<double>(h, L, false, false, L.b, S_TMP, false, 0.0, 0));
            TRY(resnorm_dd(h, L.b, L.u, nullptr, 0, nullptr, S_SUMSQ, false, 0.0, 0, 0.0));
        }
    }
    if (rel_res) {
        double v[4];
        TRY(read_scalars(h, v, 0, 4));
        *rel_res = sqrt(v[S_SUMSQ]) / sqrt(v[S_TMP]);
    }
    return BMG_OK;
}

// Reads (count, stop) back after a batch of cycles.
static bmg_status poll(bmg_solver *h, int cs[2])
{
    HIPCHK(hipMemcpyAsync(cs, h->count, 2 * sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return BMG_OK;
}

bmg_status bmg_solve(bmg_solver *h, const double *rhs, double *x, double tol, bmg_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!h || !rhs || !x) return fail(BMG_EINVAL, "NULL argument");
    if (!(tol >= 0.0)) return fail(BMG_EINVAL, "tol must be >= 0");
    const Lev<double> &L = h->L[0];
    const size_t pl0 = (size_t)(L.n + 2) * L.ld * sizeof(double);
    // a new solve: no history, no stop code left from the last one
    HIPCHK(hipMemsetAsync(h->count, 0, 2 * sizeof(int), h->st));
    // ||b|| and the initial residual; the iterate starts in L0.u (FP64) or XH
    TRY(pack_in(h, rhs, h->B0));
    TRY(pack_in(h, x, h->XH));
    HIPCHK(hipMemsetAsync(h->XL, 0, pl0, h->st));
    TRY(sumsq<double>(h, L, false, false, h->B0, S_TMP, false, 0.0, 0));
    TRY(resnorm_dd(h, h->B0, h->XH, nullptr, 0, nullptr, S_SUMSQ, false, 0.0, 0, 0.0));
    double v[S_NSCAL];
    TRY(read_scalars(h, v, 0, S_NSCAL));
    const int maxc = h->opt.max_cycles;
    if (v[S_TMP] == 0.0) {
        HIPCHK(hipMemsetAsync(h->XH, 0, pl0, h->st));
        TRY(pack_out(h, h->XH, x));
        HIPCHK(hipStreamSynchronize(h->st));
        if (info) {
            info->cycles = 0; info->rel_res = 0.0; info->rho = 0.0; info->floor_est = 0.0;
            info->t_setup_ms = h->t_setup_ms; info->t_solve_ms = ms_since(t0); info->interp_used = h->opt.interp;
            info->learned_levels_used = h->learned_used;
        }
        return BMG_OK;
    }
    double init[2] = {sqrt(v[S_TMP]), sqrt(v[S_SUMSQ]) / sqrt(v[S_TMP])};
    HIPCHK(hipMemcpyAsync(h->scal + S_BNORM, init, sizeof init, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipMemsetAsync(h->count, 0, 2 * sizeof(int), h->st));
    int cs[2] = {0, 0};
    const int every = h->opt.check_every;
    bool refining = false;
    if (!h->f32) {
        // plain V-cycles on L0.u until rel <= refine_factor * tol, then
        // refinement steps on (XH, XL); history[k] = residual after cycle k+1
        HIPCHK(hipMemcpyAsync(L.b, h->B0, pl0, hipMemcpyDeviceToDevice, h->st));
        HIPCHK(hipMemcpyAsync(L.u, h->XH, pl0, hipMemcpyDeviceToDevice, h->st));
        const double refine = h->opt.refine_factor > 0 ? h->opt.refine_factor * tol : 0.0;
        const bool pp = postpre_ok(h);
        bool pending = false;
        while (true) {
            for (int t = 0; t < every; ++t) {
                if (!refining) {
                    if (pp && pending && h->opt.graph_mode && !h->pair_off && h->tr_class < 0 && t + 1 < every) {
                        TRY(cycle_pair_graph(h, tol, maxc, refine, &pending));
                        ++t;
                    } else if (pp) {
                        TRY(cycle_and_norm_pp(h, tol, maxc, refine, &pending));
                    } else {
                        TRY(cycle_and_norm(h, tol, maxc, refine));
                    }
                } else {
                    TRY(refine_step64(h, h->stop));
                    TRY(resnorm_dd(h, h->B0, h->XH, h->XL, 2, nullptr, S_SUMSQ, true, tol, maxc, 0.0));
                }
            }
            TRY(poll(h, cs));
            if (cs[1] == 4 && !refining) {
                // the iterate becomes (XH, XL) = (u, 0); the next cycle starts
                // from zero on r = B0 - A XH (the residual just recorded)
                refining = true;
                HIPCHK(hipMemcpyAsync(h->XH, L.u, pl0, hipMemcpyDeviceToDevice, h->st));
                HIPCHK(hipMemsetAsync(h->XL, 0, pl0, h->st));
                TRY(resnorm_dd(h, h->B0, h->XH, h->XL, 2, nullptr, S_TMP, false, 0.0, 0, 0.0));
                HIPCHK(hipMemsetAsync(h->stop, 0, sizeof(int), h->st));
                continue;
            }
            if (cs[1]) break;
        }
    } else {
        // history[0] = initial residual, history[k] after correction k
        refining = true;
        const int maxe = maxc + 1;
        TRY(resnorm_dd(h, h->B0, h->XH, h->XL, 1, L.r, S_SUMSQ, true, tol, maxe, 0.0));
        while (true) {
            for (int t = 0; t < every; ++t) {
                TRY(ir_correct(h, h->stop));
                TRY(resnorm_dd(h, h->B0, h->XH, h->XL, 1, L.r, S_SUMSQ, true, tol, maxe, 0.0));
            }
            TRY(poll(h, cs));
            if (cs[1]) break;
        }
    }
    if (!refining) {
        HIPCHK(hipMemcpyAsync(h->XH, L.u, pl0, hipMemcpyDeviceToDevice, h->st));
        HIPCHK(hipMemsetAsync(h->XL, 0, pl0, h->st));
    }
    TRY(pack_out(h, h->XH, x));
    double fl = 0.0;
    if (info) {
        TRY(floor_sum(h, h->B0, h->XH));
        HIPCHK(hipMemcpyAsync(&fl, h->scal + S_FLOOR, sizeof fl, hipMemcpyDeviceToHost, h->st));
    }
    // the first and last entries of the history, and all of it into the
    // caller's array if given (no host buffer of the library's own)
    double hfirst = init[1], hlast = init[1];
    if (cs[0] > 0) {
        HIPCHK(hipMemcpyAsync(&hfirst, h->hist, sizeof(double), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipMemcpyAsync(&hlast, h->hist + (cs[0] - 1), sizeof(double), hipMemcpyDeviceToHost, h->st));
        if (info && info->history)
            HIPCHK(hipMemcpyAsync(info->history, h->hist, cs[0] * sizeof(double), hipMemcpyDeviceToHost, h->st));
    }
    HIPCHK(hipStreamSynchronize(h->st));
    const int steps = h->f32 ? std::max(cs[0] - 1, 0) : cs[0];
    if (info) {
        info->cycles = steps;
        info->rel_res = hlast;
        const double r0 = h->f32 ? hfirst : init[1];
        info->rho = steps > 0 ? pow(info->rel_res / r0, 1.0 / steps) : 0.0;
        info->floor_est = ldexp(sqrt(fl), -53) / init[0];
        info->t_setup_ms = h->t_setup_ms;
        info->t_solve_ms = ms_since(t0);
        info->interp_used = h->opt.interp;
        info->learned_levels_used = h->learned_used;
    }
    if (cs[1] == 2) return fail(BMG_EDIVERGED, "residual %.3e after %d cycles", hlast, steps);
    if (cs[1] == 3) return fail(BMG_ENOCONV, "relative residual %.3e > tol %.3e after %d cycles", hlast, tol, steps);
    return BMG_OK;
}

}  // extern "C"

// ------------------------------------------------ allocation-free solve
// The hierarchy of bmg_solve_noalloc lives in this array.  Each GPU holds its
// own copy at its own address; in host code the array's name is only a
// stand-in, so host code uses the address hipGetSymbolAddress gives for the
// current device (taken once per device, on the first call there) and never
// the name.
static __device__ __align__(256) char scratch[BMG_NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[NOALLOC_DEVICES];

// The device address of the current device's copy of scratch.
bmg_status scratch_address(char **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_DEVICES) return fail(BMG_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(BMG_EDEVICE, "no device address for the allocation-free workspace");
        g_scratch[dev] = (char *)p;
    }
    *out = g_scratch[dev];
    return BMG_OK;
}
}  // namespace

extern "C" {

bmg_status bmg_solve_noalloc(const double *stencil, int n, int kind, const bmg_options *o, const double *rhs,
                             double *x, double tol, bmg_info *info, bmg_stream stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!rhs || !x) return fail(BMG_EINVAL, "NULL argument");
    if (!(tol >= 0.0)) return fail(BMG_EINVAL, "tol must be >= 0");
    bmg_options op;
    size_t need = 0;
    TRY(check_setup(stencil, n, kind, o, &op, &need));
    if (need > BMG_NOALLOC_BYTES)
        return fail(BMG_EWORKSPACE, "n=%d needs %zu bytes of workspace; the allocation-free solve holds %zu", n,
                    need, (size_t)BMG_NOALLOC_BYTES);
    char *ws = nullptr;
    TRY(scratch_address(&ws));
    bmg_solver h;   // on the stack; its event list stays empty (no tracing)
    TRY(setup_into(&h, stencil, n, kind, op, ws, BMG_NOALLOC_BYTES, need, stream));
    h.t_setup_ms = ms_since(t0);
    return bmg_solve(&h, rhs, x, tol, info);
}

// --------------------------------------------------------- level access
// `cycles` FP64 V-cycles from x (tight n x n) on h; rho is the mean factor per
// cycle over the second half of the probe, (r_cycles / r_(cycles/2))^(2/cycles),
// which leaves out the first cycles' fast decay of the components an initial
// guess makes easy; the iterate goes to xout (tight).
static bmg_status probe(bmg_solver *h, const double *rhs, const double *x, double *xout, int cycles, double *rho)
{
    const Lev<double> &L = h->L[0];
    TRY(pack_in(h, rhs, L.b));
    TRY(pack_in(h, x, L.u));
    double v[S_NSCAL], rmid = 0.0;
    const int half = cycles / 2;
    for (int k = 1; k <= cycles; ++k) {
        TRY(cycle64(h, nullptr));
        if (k == half || k == cycles) {
            TRY(resnorm_dd(h, L.b, L.u, nullptr, 0, nullptr, S_SUMSQ, false, 0.0, 0, 0.0));
            TRY(read_scalars(h, v, 0, 4));
            if (k == half) rmid = v[S_SUMSQ];
        }
    }
    *rho = rmid > 0.0 ? pow(v[S_SUMSQ] / rmid, 1.0 / (cycles - half)) : 0.0;
    *rho = sqrt(*rho);   // the sums are of squares
    TRY(pack_out(h, L.u, xout));
    return BMG_OK;
}

bmg_status bmg_solve_select(bmg_solver *learned, bmg_solver *boxmg, const double *rhs, double *x, double tol,
                            int probe_cycles, bmg_info *info, int *used, double *rho)
{
    if (!learned || !boxmg || !rhs || !x || !used || !rho) return fail(BMG_EINVAL, "NULL argument");
    if (learned->n != boxmg->n) return fail(BMG_EINVAL, "the two hierarchies have different sizes");
    if (learned->opt.precision != BMG_FP64 || boxmg->opt.precision != BMG_FP64)
        return fail(BMG_EINVAL, "the probe compares FP64 hierarchies");
    if (learned->opt.interp != BMG_INTERP_LEARNED || boxmg->opt.interp != BMG_INTERP_BOXMG)
        return fail(BMG_EINVAL, "expected a learned and an operator-induced hierarchy");
    if (probe_cycles == 0) probe_cycles = 8;
    if (probe_cycles < 2 || probe_cycles > 1000) return fail(BMG_EINVAL, "probe_cycles=%d out of range", probe_cycles);
    // the BoxMG probe reads x first and leaves its iterate in its XH buffer
    // (tight n x n); the learned probe then overwrites x with its own
    double *scratch = boxmg->XH;
    TRY(probe(boxmg, rhs, x, scratch, probe_cycles, &rho[1]));
    HIPCHK(hipStreamSynchronize(boxmg->st));
    TRY(probe(learned, rhs, x, x, probe_cycles, &rho[0]));
    // the learned probe's write of x completes before any other stream uses x
    HIPCHK(hipStreamSynchronize(learned->st));
    if (rho[0] > rho[1]) {
        *used = BMG_INTERP_BOXMG;
        HIPCHK(hipMemcpyAsync(x, scratch, (size_t)boxmg->n * boxmg->n * sizeof(double), hipMemcpyDeviceToDevice,
                              boxmg->st));
        HIPCHK(hipStreamSynchronize(boxmg->st));
        const bmg_status s = bmg_solve(boxmg, rhs, x, tol, info);
        if (info) {
            info->cycles += probe_cycles;
            info->interp_used = BMG_INTERP_BOXMG;
        }
        return s;
    }
    // the learned hierarchy continues in chunks of WATCH cycles; a chunk whose
    // factor exceeds the BoxMG probe's hands the iterate to BoxMG
    constexpr int WATCH = 16;
    *used = BMG_INTERP_LEARNED;
    const int maxc = learned->opt.max_cycles;
    int done = probe_cycles;
    bmg_status s = BMG_ENOCONV;
    double *hist = info ? info->history : nullptr;
    bmg_info ci{};
    // each chunk's history goes after the previous chunks' (the caller's
    // array holds max_cycles + 1 entries, the cycles after the probes)
    while (done < maxc + probe_cycles) {
        learned->opt.max_cycles = std::min(WATCH, maxc + probe_cycles - done);
        ci = bmg_info{};
        ci.history = hist ? hist + (done - probe_cycles) : nullptr;
        s = bmg_solve(learned, rhs, x, tol, &ci);
        learned->opt.max_cycles = maxc;
        done += ci.cycles;
        if (s != BMG_ENOCONV) break;
        if (ci.rho > rho[1]) {
            *used = BMG_INTERP_BOXMG;
            const int left = maxc + probe_cycles - done;
            if (left <= 0) break;
            const int keep = boxmg->opt.max_cycles;
            boxmg->opt.max_cycles = std::min(keep, left);
            ci = bmg_info{};
            ci.history = hist ? hist + (done - probe_cycles) : nullptr;
            s = bmg_solve(boxmg, rhs, x, tol, &ci);
            boxmg->opt.max_cycles = keep;
            done += ci.cycles;
            break;
        }
    }
    if (info) {
        double *h0 = info->history;
        *info = ci;
        info->history = h0;
        info->cycles = done;
        info->interp_used = *used;
    }
    return s;
}

bmg_status bmg_num_levels(const bmg_solver *h, int *nlev)
{
    if (!h || !nlev) return fail(BMG_EINVAL, "NULL argument");
    *nlev = h->nlev;
    return BMG_OK;
}

bmg_status bmg_level_n(const bmg_solver *h, int level, int *n)
{
    if (!h || !n) return fail(BMG_EINVAL, "NULL argument");
    if (level < 0 || level >= h->nlev) return fail(BMG_EINVAL, "level %d out of range", level);
    *n = h->L[level].n;
    return BMG_OK;
}

// Resolves (level, field) to a device array, its element size, pitch, row
// count and row width of the tight layout.
static bmg_status locate(bmg_solver *h, int level, int field, char **ptr, size_t *es, size_t *pitch,
                         size_t *rows, size_t *width)
{
    if (!h) return fail(BMG_EINVAL, "NULL handle");
    if (field == BMG_F_COARSE_LD) {
        const size_t cnt = (size_t)h->band.m * (h->band.nc + 1) + h->band.m;
        *ptr = (char *)h->Lb; *es = 8; *pitch = cnt * 8; *rows = 1; *width = cnt;
        return BMG_OK;
    }
    if (field == BMG_F_XLO) {
        *ptr = (char *)h->XL; *es = 8; *pitch = (size_t)h->L[0].ld * 8;
        *rows = h->L[0].n + 2; *width = h->L[0].n + 2;
        return BMG_OK;
    }
    if (level < 0 || level >= h->nlev) return fail(BMG_EINVAL, "level %d out of range", level);
    const bool f32 = field >= BMG_F_U32;
    if (f32 && !h->f32) return fail(BMG_EINVAL, "FP32 fields need precision BMG_FP32_IR");
    const int fb = f32 ? field - BMG_F_U32 : field;
    const Lev<double> &L = h->L[level];
    const Lev<float> &F = h->L32[level];
    void *p = nullptr;
    switch (fb) {
    case BMG_F_U: p = f32 ? (void *)F.u : (void *)L.u; break;
    case BMG_F_B: p = f32 ? (void *)F.b : (void *)L.b; break;
    case BMG_F_R: p = f32 ? (void *)F.r : (void *)L.r; break;
    case BMG_F_AO: p = f32 ? (void *)F.O : (void *)L.O; break;
    case BMG_F_AW: p = f32 ? (void *)F.W : (void *)L.W; break;
    case BMG_F_AS: p = f32 ? (void *)F.S : (void *)L.S; break;
    case BMG_F_ASW: p = f32 ? (void *)F.SW : (void *)L.SW; break;
    case BMG_F_ANW: p = f32 ? (void *)F.NW : (void *)L.NW; break;
    case BMG_F_CI: {
        if (level + 1 >= h->nlev) return fail(BMG_EINVAL, "the coarsest level has no weights");
        p = f32 ? (void *)h->C32[level].p : (void *)h->C[level].p;
        const int nc = h->L[level + 1].n;
        *ptr = (char *)p; *es = f32 ? 4 : 8; *pitch = (size_t)h->C[level].ld * *es;
        *rows = 8 * (size_t)(nc + 2); *width = nc + 2;
        return BMG_OK;
    }
    default: return fail(BMG_EINVAL, "unknown field %d", field);
    }
    if (!p) return fail(BMG_EINVAL, "field %d does not exist on level %d", field, level);
    *ptr = (char *)p; *es = f32 ? 4 : 8; *pitch = (size_t)L.ld * *es; *rows = L.n + 2; *width = L.n + 2;
    return BMG_OK;
}

// The level operator in the input layout of bmg_setup.
static __global__ void k_export_stencil(Lev<double> L, bool nine, double *__restrict__ st)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const size_t ld = L.ld, p = (size_t)j * ld + i;
    const size_t o = ((size_t)(j - 1) * L.n + (i - 1)) * (nine ? 9 : 5);
    if (nine) {
        st[o + 0] = L.SW[p];
        st[o + 1] = L.S[p];
        st[o + 2] = L.NW[p + 1 - ld];
        st[o + 3] = L.W[p];
        st[o + 4] = L.O[p];
        st[o + 5] = L.W[p + 1];
        st[o + 6] = L.NW[p];
        st[o + 7] = L.S[p + ld];
        st[o + 8] = L.SW[p + ld + 1];
    } else {
        st[o + 0] = L.S[p];
        st[o + 1] = L.W[p];
        st[o + 2] = L.O[p];
        st[o + 3] = L.W[p + 1];
        st[o + 4] = L.S[p + ld];
    }
}

bmg_status bmg_export(bmg_solver *h, int level, int field, void *dst)
{
    if (field == BMG_F_STENCIL) {
        if (!h || !dst) return fail(BMG_EINVAL, "NULL argument");
        if (level < 0 || level >= h->nlev) return fail(BMG_EINVAL, "level %d out of range", level);
        const Lev<double> &L = h->L[level];
        hipLaunchKernelGGL(k_export_stencil, grid2(L.n, L.n, B2), B2, 0, h->st, L, h->nine[level], (double *)dst);
        LAUNCHCHK();
        return BMG_OK;
    }
    char *p; size_t es, pitch, rows, width;
    TRY(locate(h, level, field, &p, &es, &pitch, &rows, &width));
    if (!dst) return fail(BMG_EINVAL, "dst is NULL");
    HIPCHK(hipMemcpy2DAsync(dst, width * es, p, pitch, width * es, rows, hipMemcpyDeviceToDevice, h->st));
    return BMG_OK;
}

bmg_status bmg_import(bmg_solver *h, int level, int field, const void *src)
{
    char *p; size_t es, pitch, rows, width;
    TRY(locate(h, level, field, &p, &es, &pitch, &rows, &width));
    if (!src) return fail(BMG_EINVAL, "src is NULL");
    HIPCHK(hipMemcpy2DAsync(p, pitch, src, width * es, width * es, rows, hipMemcpyDeviceToDevice, h->st));
    return BMG_OK;
}

}  // extern "C"

template <typename T>
static bmg_status step_t(bmg_solver *h, int l, int step, int arg)
{
    const Lev<T> &F = lev<T>(h, l);
    const bool last = l == h->nlev - 1;
    if (last && step != BMG_STEP_SMOOTH && step != BMG_STEP_RESIDUAL && step != BMG_STEP_COARSE)
        return fail(BMG_EINVAL, "step %d needs a coarser level below level %d", step, l);
    switch (step) {
    case BMG_STEP_SMOOTH: return smooth<T>(h, F, h->nine[l], arg, nullptr, l);
    case BMG_STEP_RESIDUAL: return residual<T>(h, F, h->nine[l], nullptr);
    case BMG_STEP_RESTRICT: return restrict_<T>(h, F, wts<T>(h, l), lev<T>(h, l + 1), nullptr);
    case BMG_STEP_INTERP: return interp<T>(h, F, wts<T>(h, l), lev<T>(h, l + 1), nullptr);
    case BMG_STEP_COARSE:
        if (!last) return fail(BMG_EINVAL, "the direct solve runs on the coarsest level only");
        return coarse<T>(h, F, nullptr);
    case BMG_STEP_PRE:
    case BMG_STEP_POST:
        if (h->opt.smoother != BMG_SMOOTH_POINT) return fail(BMG_EINVAL, "the fused passes relax pointwise");
        return step == BMG_STEP_PRE ? fused_pre<T>(h, l, arg, nullptr) : fused_post<T>(h, l, arg, nullptr);
    default: return fail(BMG_EINVAL, "unknown step %d", step);
    }
}

extern "C" bmg_status bmg_step(bmg_solver *h, int level, int step, int arg, int fp32)
{
    if (!h) return fail(BMG_EINVAL, "NULL handle");
    if (level < 0 || level >= h->nlev) return fail(BMG_EINVAL, "level %d out of range", level);
    if (arg < 0 || arg > 64) return fail(BMG_EINVAL, "step argument %d out of range", arg);
    if (fp32) {
        if (!h->f32) return fail(BMG_EINVAL, "FP32 steps need precision BMG_FP32_IR");
        return step_t<float>(h, level, step, arg);
    }
    return step_t<double>(h, level, step, arg);
}

extern "C" {

bmg_status bmg_trace_enable(bmg_solver *h, int kclass, int level, int on)
{
    if (!h) return fail(BMG_EINVAL, "NULL handle");
    if (kclass < BMG_TRACE_SMOOTH || kclass > BMG_TRACE_POSTPRE) return fail(BMG_EINVAL, "unknown class");
    h->tr_class = on ? kclass : -1;
    h->tr_level = level;
    h->tr_used = 0;
    h->tr_bytes = 0.0;
    return BMG_OK;
}

bmg_status bmg_trace_read(bmg_solver *h, int *launches, double *total_ms, double *bytes)
{
    if (!h || !launches || !total_ms) return fail(BMG_EINVAL, "NULL argument");
    HIPCHK(hipStreamSynchronize(h->st));
    double tot = 0.0;
    for (int t = 0; t + 1 < h->tr_used; t += 2) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->tr_ev[t], h->tr_ev[t + 1]));
        tot += ms;
    }
    *launches = h->tr_used / 2;
    *total_ms = tot;
    if (bytes) *bytes = h->tr_bytes;
    h->tr_used = 0;
    h->tr_bytes = 0.0;
    return BMG_OK;
}

}  // extern "C"

// ------------------------------------------------------------ block solves
// A block is a second view of a hierarchy: `hb` shares the operators, weights
// and coarsest factor of the parent handle and points its iterate and
// right-hand-side arrays at k planes per level (nrhs = k), so the fused cycle
// code runs all of them in each launch; view[j] is right-hand side j alone
// (nrhs = 1), on which the per-right-hand-side steps of bmg_solve run
// unchanged.  Each fused pass swaps a level's iterate buffers, twice per cycle,
// so between cycles every view's pointers are the block's again.
struct bmg_block {
    bmg_solver *parent = nullptr;
    int k = 0;
    bmg_solver hb;
    std::vector<bmg_solver> view;
    int *mode = nullptr;        // device: each right-hand side's state in the solve
};

namespace {

bmg_status block_check(const bmg_solver *h, int k)
{
    if (!h) return fail(BMG_EINVAL, "NULL handle");
    if (k < 1 || k > 4096) return fail(BMG_EINVAL, "k=%d right-hand sides must be in [1, 4096]", k);
    if (h->opt.precision != BMG_FP64) return fail(BMG_EINVAL, "block solves run FP64 hierarchies");
    if (h->opt.kernels != BMG_KERNELS_FUSED || h->opt.smoother != BMG_SMOOTH_POINT)
        return fail(BMG_EINVAL, "block solves need the fused kernels (point relaxation)");
    if (h->opt.nu1 < 1 || h->opt.nu1 > 3 || h->opt.nu2 < 1 || h->opt.nu2 > 2)
        return fail(BMG_EINVAL, "block solves need 1 <= nu1 <= 3 and 1 <= nu2 <= 2");
    return BMG_OK;
}

// Walks the block's workspace; with base == nullptr it only measures.
size_t block_plan(const bmg_solver *h, int k, char *base, bmg_block *B)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + ALIGN - 1) & ~(ALIGN - 1);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    // planes rounded to ALIGN so that every right-hand side's plane is aligned
    auto plane = [&](int l) { return (((size_t)(h->L[l].n + 2) * h->L[l].ld * 8 + ALIGN - 1) & ~(ALIGN - 1)) / 8; };
    double *u[MAXL], *ua[MAXL], *b[MAXL];
    for (int l = 0; l < h->nlev; ++l) {
        u[l] = (double *)take(k * plane(l) * 8);
        ua[l] = (double *)take(k * plane(l) * 8);
        b[l] = (double *)take(k * plane(l) * 8);
    }
    const size_t p0 = plane(0);
    double *B0 = (double *)take(k * p0 * 8);
    double *XH = (double *)take(k * p0 * 8);
    double *XL = (double *)take(k * p0 * 8);
    double *part = (double *)take((size_t)k * NPART * 8);
    double *scal = (double *)take((size_t)k * S_NSCAL * 8);
    double *hist = (double *)take((size_t)k * h->hist_cap * 8);
    int *cnt = (int *)take((size_t)k * 2 * sizeof(int));
    int *mode = (int *)take((size_t)k * sizeof(int));
    if (B) {
        B->mode = mode;
        bmg_solver &v = B->hb;
        v = *h;
        v.tr_ev.clear();
        v.tr_class = v.tr_level = -1;
        v.tr_used = 0;
        v.tr_bytes = v.tr_pending = 0.0;
        v.ws = nullptr;
        v.ws_bytes = 0;
        v.nrhs = k;
        v.kstop = 2;
        v.kpart = NPART;
        for (int l = 0; l < h->nlev; ++l) {
            v.ks[l] = plane(l);
            v.L[l].u = u[l];
            v.L[l].b = b[l];
            v.L[l].r = nullptr;   // the fused passes keep residuals on chip
            v.ualt[l] = ua[l];
        }
        v.B0 = B0;
        v.XH = XH;
        v.XL = XL;
        v.part = part;
        v.scal = scal;
        v.hist = hist;
        v.count = cnt;
        v.stop = cnt + 1;
        B->view.assign(k, v);
        for (int j = 0; j < k; ++j) {
            bmg_solver &w = B->view[j];
            w.nrhs = 1;
            w.kstop = w.kpart = 0;
            for (int l = 0; l < h->nlev; ++l) {
                w.ks[l] = 0;
                w.L[l].u = u[l] + j * v.ks[l];
                w.L[l].b = b[l] + j * v.ks[l];
                w.ualt[l] = ua[l] + j * v.ks[l];
            }
            w.B0 = B0 + j * p0;
            w.XH = XH + j * p0;
            w.XL = XL + j * p0;
            w.part = part + (size_t)j * NPART;
            w.scal = scal + (size_t)j * S_NSCAL;
            w.hist = hist + (size_t)j * h->hist_cap;
            w.count = cnt + 2 * j;
            w.stop = cnt + 2 * j + 1;
        }
    }
    return (off + ALIGN - 1) & ~(ALIGN - 1);
}

}  // namespace

extern "C" {

bmg_status bmg_block_workspace_bytes(const bmg_solver *h, int k, size_t *bytes)
{
    TRY(block_check(h, k));
    if (!bytes) return fail(BMG_EINVAL, "NULL argument");
    *bytes = block_plan(h, k, nullptr, nullptr);
    return BMG_OK;
}

bmg_status bmg_block_create(bmg_block **out, bmg_solver *h, int k, void *workspace, size_t bytes)
{
    if (!out) return fail(BMG_EINVAL, "NULL argument");
    *out = nullptr;
    TRY(block_check(h, k));
    if (!workspace) return fail(BMG_EINVAL, "NULL workspace");
    if ((uintptr_t)workspace % ALIGN) return fail(BMG_EINVAL, "workspace not %zu-byte aligned", ALIGN);
    const size_t need = block_plan(h, k, nullptr, nullptr);
    if (bytes < need) return fail(BMG_EWORKSPACE, "block workspace %zu < %zu bytes", bytes, need);
    bmg_block *B = new bmg_block;
    B->parent = h;
    B->k = k;
    block_plan(h, k, (char *)workspace, B);
    *out = B;
    return BMG_OK;
}

bmg_status bmg_block_destroy(bmg_block *B)
{
    if (!B) return BMG_OK;
    for (hipEvent_t e : B->hb.tr_ev) (void)hipEventDestroy(e);
    delete B;
    return BMG_OK;
}

bmg_status bmg_block_trace_enable(bmg_block *B, int kclass, int level, int on)
{
    if (!B) return fail(BMG_EINVAL, "NULL handle");
    return bmg_trace_enable(&B->hb, kclass, level, on);
}

bmg_status bmg_block_trace_read(bmg_block *B, int *launches, double *total_ms, double *bytes)
{
    if (!B) return fail(BMG_EINVAL, "NULL handle");
    return bmg_trace_read(&B->hb, launches, total_ms, bytes);
}

bmg_status bmg_block_solve(bmg_block *B, const double *rhs, double *x, double tol, bmg_info *info,
                           bmg_status *status)
{
    if (!B || !rhs || !x) return fail(BMG_EINVAL, "NULL argument");
    if (!(tol >= 0.0)) return fail(BMG_EINVAL, "tol must be >= 0");
    bmg_solver *hb = &B->hb;
    const int K = B->k;
    const Lev<double> &L = hb->L[0];
    const size_t n2 = (size_t)L.n * L.n;
    const size_t pl0 = (size_t)(L.n + 2) * L.ld * sizeof(double);
    const int maxc = hb->opt.max_cycles;
    const double refine = hb->opt.refine_factor > 0 ? hb->opt.refine_factor * tol : 0.0;
    enum { PLAIN, REFINING, ZERO };
    std::vector<int> mode(K, PLAIN), cs(2 * K, 0);
    std::vector<double> sc((size_t)K * S_NSCAL), init(2 * (size_t)K, 0.0);
    // each right-hand side's ||b|| and initial residual, as bmg_solve starts
    HIPCHK(hipMemsetAsync(hb->count, 0, 2 * K * sizeof(int), hb->st));
    for (int j = 0; j < K; ++j) {
        bmg_solver *v = &B->view[j];
        TRY(pack_in(v, rhs + j * n2, v->B0));
        TRY(pack_in(v, x + j * n2, v->XH));
        HIPCHK(hipMemsetAsync(v->XL, 0, pl0, hb->st));
        TRY(sumsq<double>(v, v->L[0], false, false, v->B0, S_TMP, false, 0.0, 0));
        TRY(resnorm_dd(v, v->B0, v->XH, nullptr, 0, nullptr, S_SUMSQ, false, 0.0, 0, 0.0));
    }
    TRY(read_scalars(hb, sc.data(), 0, K * S_NSCAL));
    for (int j = 0; j < K; ++j) {
        bmg_solver *v = &B->view[j];
        const double *s = &sc[(size_t)j * S_NSCAL];
        if (s[S_TMP] == 0.0) {
            // a zero right-hand side: x = 0 after 0 cycles; its stop flag keeps
            // every launch of the block from touching it
            mode[j] = ZERO;
            cs[2 * j + 1] = 1;
            HIPCHK(hipMemsetAsync(v->XH, 0, pl0, hb->st));
            continue;
        }
        init[2 * j] = sqrt(s[S_TMP]);
        init[2 * j + 1] = sqrt(s[S_SUMSQ]) / sqrt(s[S_TMP]);
        HIPCHK(hipMemcpyAsync(v->scal + S_BNORM, &init[2 * j], 2 * sizeof(double), hipMemcpyHostToDevice, hb->st));
        HIPCHK(hipMemcpyAsync(v->L[0].b, v->B0, pl0, hipMemcpyDeviceToDevice, hb->st));
        HIPCHK(hipMemcpyAsync(v->L[0].u, v->XH, pl0, hipMemcpyDeviceToDevice, hb->st));
    }
    HIPCHK(hipMemcpyAsync(hb->count, cs.data(), 2 * K * sizeof(int), hipMemcpyHostToDevice, hb->st));
    HIPCHK(hipMemcpyAsync(B->mode, mode.data(), K * sizeof(int), hipMemcpyHostToDevice, hb->st));
    HIPCHK(hipStreamSynchronize(hb->st));   // init[], cs[] and mode[] are read by the copies above
    // the per-right-hand-side steps of a cycle run as one launch each over the
    // right-hand sides in the state they apply to
    const size_t p0 = hb->ks[0];            // elements between right-hand sides' fine planes
    auto fan = [&](int want) {
        RhsFan F;
        F.nrhs = K;
        F.mode = B->mode;
        F.want = want;
        F.kl = hb->ks[0];
        F.kx = p0;
        F.kpart = NPART;
        F.kscal = S_NSCAL;
        F.khist = hb->hist_cap;
        F.kcnt = 2;
        return F;
    };
    const int nb = std::min(NPART_ROWS, L.n);
    const int every = hb->opt.check_every;
    while (true) {
        const bool any_plain = std::count(mode.begin(), mode.end(), (int)PLAIN) > 0;
        const bool any_ref = std::count(mode.begin(), mode.end(), (int)REFINING) > 0;
        for (int t = 0; t < every; ++t) {
            // one V-cycle of every running right-hand side (plain: on (b, u);
            // refining: on (r, 0)); stopped ones return at once
            TRY(fused_vcycle(hb, hb->stop, true));
            if (any_plain) {
                if (hb->norm_parts > 0) {
                    hipLaunchKernelGGL(k_sumsq_final_fan, dim3(K), dim3(1024), 0, hb->st, (const double *)hb->part,
                                       hb->norm_parts, hb->scal + S_SUMSQ, hb->hist, hb->count,
                                       (const double *)(hb->scal + S_BNORM), tol, maxc, refine, fan(PLAIN));
                    LAUNCHCHK();
                } else {
                    for (int j = 0; j < K; ++j) {
                        bmg_solver *v = &B->view[j];
                        if (mode[j] == PLAIN)
                            TRY(resnorm_dd(v, v->L[0].b, v->L[0].u, nullptr, 0, nullptr, S_SUMSQ, true, tol, maxc,
                                           refine));
                    }
                }
            }
            if (any_ref) {
                // (XH, XL) += u, then r = B0 - A (XH + XL) -> b and 0 -> u
                dim3 g = grid2(L.n, L.n, B2);
                g.z = K;
                hipLaunchKernelGGL(k_dd_update_fan, g, B2, 0, hb->st, L, hb->XH, hb->XL, (const int *)hb->stop,
                                   fan(REFINING));
                if (hb->nine[0])
                    hipLaunchKernelGGL((k_resid_dd_fan<true, 2>), dim3(nb * K), dim3(256), 0, hb->st, L,
                                       (const double *)hb->B0, (const double *)hb->XH, (const double *)hb->XL,
                                       hb->part, (const int *)hb->stop, fan(REFINING));
                else
                    hipLaunchKernelGGL((k_resid_dd_fan<false, 2>), dim3(nb * K), dim3(256), 0, hb->st, L,
                                       (const double *)hb->B0, (const double *)hb->XH, (const double *)hb->XL,
                                       hb->part, (const int *)hb->stop, fan(REFINING));
                hipLaunchKernelGGL(k_sumsq_final_fan, dim3(K), dim3(1024), 0, hb->st, (const double *)hb->part, nb,
                                   hb->scal + S_SUMSQ, hb->hist, hb->count, (const double *)(hb->scal + S_BNORM),
                                   tol, maxc, 0.0, fan(REFINING));
                LAUNCHCHK();
            }
        }
        HIPCHK(hipMemcpyAsync(cs.data(), hb->count, 2 * K * sizeof(int), hipMemcpyDeviceToHost, hb->st));
        HIPCHK(hipStreamSynchronize(hb->st));
        bool running = false, switched = false;
        for (int j = 0; j < K; ++j) {
            bmg_solver *v = &B->view[j];
            if (mode[j] == PLAIN && cs[2 * j + 1] == 4) {
                // as bmg_solve: (XH, XL) = (u, 0), the next cycle starts from
                // zero on r = B0 - A XH
                mode[j] = REFINING;
                HIPCHK(hipMemcpyAsync(v->XH, v->L[0].u, pl0, hipMemcpyDeviceToDevice, hb->st));
                HIPCHK(hipMemsetAsync(v->XL, 0, pl0, hb->st));
                TRY(resnorm_dd(v, v->B0, v->XH, v->XL, 2, nullptr, S_TMP, false, 0.0, 0, 0.0));
                HIPCHK(hipMemsetAsync(v->stop, 0, sizeof(int), hb->st));
                running = switched = true;
            } else if (mode[j] != ZERO && cs[2 * j + 1] == 0) {
                running = true;
            }
        }
        if (switched) {
            HIPCHK(hipMemcpyAsync(B->mode, mode.data(), K * sizeof(int), hipMemcpyHostToDevice, hb->st));
            HIPCHK(hipStreamSynchronize(hb->st));
        }
        if (!running) break;
    }
    bmg_status first = BMG_OK;
    std::vector<double> hist((size_t)hb->hist_cap);
    for (int j = 0; j < K; ++j) {
        bmg_solver *v = &B->view[j];
        if (mode[j] == PLAIN) {
            HIPCHK(hipMemcpyAsync(v->XH, v->L[0].u, pl0, hipMemcpyDeviceToDevice, hb->st));
            HIPCHK(hipMemsetAsync(v->XL, 0, pl0, hb->st));
        }
        TRY(pack_out(v, v->XH, x + j * n2));
        bmg_status sj = BMG_OK;
        if (mode[j] == ZERO) {
            if (info) { info[j].cycles = 0; info[j].rel_res = 0.0; info[j].rho = 0.0; }
        } else {
            const int c = cs[2 * j];
            HIPCHK(hipMemcpyAsync(hist.data(), v->hist, c * sizeof(double), hipMemcpyDeviceToHost, hb->st));
            HIPCHK(hipStreamSynchronize(hb->st));
            if (info) {
                info[j].cycles = c;
                info[j].rel_res = c > 0 ? hist[c - 1] : init[2 * j + 1];
                info[j].rho = c > 0 ? pow(info[j].rel_res / init[2 * j + 1], 1.0 / c) : 0.0;
                if (info[j].history) memcpy(info[j].history, hist.data(), c * sizeof(double));
            }
            if (cs[2 * j + 1] == 2) sj = BMG_EDIVERGED;
            if (cs[2 * j + 1] == 3) sj = BMG_ENOCONV;
            if (sj != BMG_OK && first == BMG_OK) {
                first = sj;
                fail(sj, "right-hand side %d: relative residual %.3e after %d cycles", j, c > 0 ? hist[c - 1] : 0.0, c);
            }
        }
        if (status) status[j] = sj;
    }
    HIPCHK(hipStreamSynchronize(hb->st));
    return first;
}

}  // extern "C"
