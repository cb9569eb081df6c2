/*
 * bmg.h - C interface of the MI355X (gfx950) black-box multigrid library.
 *
 * The library solves the stencil system A u = b that a standard
 * finite-difference discretisation of the 2D diffusion problem
 * -div(k grad u) = f gives on a vertex-centred grid (Section 2, Eq. 1 of the
 * paper), with the BoxMG V-cycle of Section 2 and Fig. vcycle_flowchart:
 * Gauss-Seidel relaxation, residual, restriction, recursion to a direct solve
 * on the coarsest grid, interpolation, relaxation.  Coarse operators are built
 * by local stencil operations (Section 2), restriction follows
 * Fig. restrict_kernel and the stencil of each point is the nine-point stencil
 * of Fig. stencil_operator.  Every step runs in hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *  - Grids: interior n x n with n = 2^m - 1, m >= 2; the mesh width is
 *    h = 1/(n+1); level l has n_l = 2^(m-l) - 1 down to the coarsest n_L
 *    (bmg_options.coarsest_n, 3 by default).
 *  - Pointers are DEVICE pointers unless the comment says "host".
 *  - Work is enqueued on the stream given at set-up (NULL = the null stream);
 *    entry points that return a number to the host synchronise that stream.
 *  - Kernels never allocate: the caller supplies one workspace buffer of the
 *    size bmg_workspace_bytes() reports.  The library keeps pointers into it
 *    and into nothing else.
 *  - Status codes only: no entry point throws or aborts; a failed call leaves
 *    a one-line description for bmg_last_error() (per host thread).
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef BMG_H
#define BMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bmg_solver bmg_solver;
typedef void *bmg_stream; /* a hipStream_t */

typedef enum {
    BMG_OK = 0,
    BMG_EINVAL = -1,      /* bad argument: size, pointer, option, stencil value */
    BMG_EBREAKDOWN = -2,  /* interpolation denominator or coarse pivot <= 0 */
    BMG_ENOCONV = -3,     /* max_cycles reached before tol */
    BMG_EDIVERGED = -4,   /* residual grew by 1e3 or became non-finite */
    BMG_EDEVICE = -5,     /* a HIP runtime call failed */
    BMG_EWORKSPACE = -6   /* workspace missing, too small or misaligned */
} bmg_status;

enum { BMG_STENCIL_5PT = 5, BMG_STENCIL_9PT = 9 };
enum { BMG_FP64 = 0, BMG_FP32_IR = 1 };
enum { BMG_KERNELS_BASIC = 0, BMG_KERNELS_FUSED = 1 };
enum { BMG_INTERP_BOXMG = 0, BMG_INTERP_LEARNED = 1 };
enum { BMG_SMOOTH_POINT = 0, BMG_SMOOTH_LINE = 1 };

typedef struct bmg_net bmg_net;   /* learned interpolation network, see below */

typedef struct {
    int nu1;         /* pre-smoothing sweeps (default 2) */
    int nu2;         /* post-smoothing sweeps (default 1) */
    int max_cycles;  /* cycle (or refinement step) limit of bmg_solve (default 100) */
    int precision;   /* BMG_FP64, or BMG_FP32_IR: FP32 V-cycle inside FP64
                        iterative refinement (default BMG_FP64) */
    int kernels;     /* BMG_KERNELS_FUSED (default) or BMG_KERNELS_BASIC: one
                        launch per colour and per step, for comparison */
    int check_every; /* bmg_solve reads the residual history back every this many
                        cycles; cycles past convergence are skipped on the device,
                        so the iterates do not depend on it (default 8) */
    int refine_factor; /* FP64: once the relative residual is <= refine_factor *
                        tol, the iterate becomes a double-FP64 pair (x, x_lo)
                        and each cycle is one refinement step with an accurate
                        residual, which converges below the residual floor of
                        FP64 vectors; 0 = never (default 16) */
    int tile_rows;   /* grid rows per workgroup tile of the fused passes
                        (even, 0 = a measured default for each level size) */
    int interp;      /* BMG_INTERP_BOXMG (default): operator-induced weights on
                        every level; BMG_INTERP_LEARNED: the weights of levels
                        l < learned_levels come from the network `net` */
    int learned_levels; /* levels with learned weights (0 = all) */
    bmg_net *net;    /* network of BMG_INTERP_LEARNED (not owned); it must
                        outlive the set-up call only */
    int smoother;    /* BMG_SMOOTH_POINT (default): four-colour point
                        Gauss-Seidel; BMG_SMOOTH_LINE: alternating zebra line
                        Gauss-Seidel (the "Line" relaxation of Fig.
                        vcycle_flowchart): x-lines odd then even, then y-lines
                        odd then even, each line's tridiagonal system solved
                        exactly with a factor formed at set-up.  FP64 only; the
                        cycle then runs one launch per step (kernels is
                        ignored) */
    int coarsest_n;  /* points per side of the coarsest level, which is solved
                        directly (Fig. vcycle_flowchart: Cholesky) with the
                        square-root-free Cholesky factor of its band matrix
                        (lexicographic unknowns, half-bandwidth coarsest_n + 1):
                        2^k - 1 with 3 <= coarsest_n <= min(n, 63); 0 = 3 */
    int persistent_below_n; /* coarse levels of at most this many points per
                        side (below the fine level) run as one persistent
                        one-workgroup launch per cycle: 2^k - 1 <= 63, or 1 for
                        none; 0 = 63 */
    int square_tiles_below_n; /* nine-point levels of at most this many points
                        per side run their fused pre and post passes with one
                        workgroup per 32 x 32 square tile, every sweep of the
                        pass inside the tile's LDS copy (one right-hand side):
                        2^k - 1, or 1 for none; 0 = 511 */
    int graph_mode;  /* 1: bmg_solve's plain FP64 cycles on the fused fine-level
                        schedule run as replays of a HIP graph of two cycles,
                        captured on the solve's stream at its first use (one
                        graph launch in place of about 26 kernel launches); the
                        results are those of the launches, bit for bit.  Not
                        used while a trace is enabled.  0 (default): direct
                        launches */
} bmg_options;

typedef struct {
    int cycles;       /* V-cycles (FP64) or refinement steps (FP32_IR) performed */
    double rel_res;   /* final ||b - A x||_2 / ||b||_2 */
    double rho;       /* geometric-mean reduction factor per cycle over the run */
    double *history;  /* host, caller-owned, max_cycles+1 entries, or NULL:
                         FP64: history[k] = relative residual after cycle k+1;
                         FP32_IR: history[0] is the initial relative residual,
                         history[k] the one after correction k */
    double floor_est; /* eps * || |A| |x| + |b| ||_2 / ||b||_2 for the returned
                         x (eps = 2^-53): the scale of the relative residual
                         that rounding x to FP64 alone can leave */
    double t_setup_ms; /* host wall time of the handle's bmg_setup */
    double t_solve_ms; /* host wall time of this call */
    int interp_used;  /* BMG_INTERP_BOXMG or BMG_INTERP_LEARNED: the weights of
                         the hierarchy that produced x */
    int learned_levels_used; /* levels of that hierarchy whose weights came from
                         the network (0 for BoxMG's).  A learned set-up stops
                         using the network above a level on whose coarse
                         operator BoxMG's formula finds a denominator <= 0: that
                         level takes BoxMG's weights and its coarse operator is
                         formed again, and so are all levels below it */
} bmg_info;

/* Fills *o with the defaults above.  Host only. */
bmg_status bmg_default_options(bmg_options *o);

/* Bytes of device workspace bmg_setup needs for an n x n grid of the given
 * stencil kind (5 or 9) and options (o may be NULL for the defaults).  The
 * workspace must be 256-byte aligned.  Host only; no device call. */
bmg_status bmg_workspace_bytes(int n, int kind, const bmg_options *o, size_t *bytes);

/* Discretisation of -div(k grad u) = f (Section 2, Eq. 1) on the n x n
 * interior grid, vertex-centred, with cell-constant k: the coupling across the
 * dual-cell face between two neighbouring vertices is minus the mean of the two
 * cells sharing that grid edge, the centre is minus the sum of the four
 * couplings (taken before couplings to the Dirichlet boundary are set to zero),
 * and the right-hand side is h^2 f.
 *   k:       (n+1) x (n+1) cell coefficients, row-major, k[jc][ic], positive;
 *   f:       n x n source, row-major, f[j-1][i-1];
 *   stencil: out, n x n x 5 in the order S, W, O, E, N (signed matrix entries);
 *   rhs:     out, n x n.
 * Enqueued on `stream`; no synchronisation.  BMG_EINVAL on a bad n or NULL. */
bmg_status bmg_discretize(const double *k, const double *f, int n, double *stencil,
                          double *rhs, bmg_stream stream);

/* Builds the multigrid hierarchy of the symmetric stencil operator (Section 2:
 * coarse operators through local stencil operations):
 *   per level, operator-induced interpolation weights (collapsed stencil, with
 *   positive off-diagonal entries moved onto the diagonal before the collapse),
 *   stored as the eight planes LNE, LA, LNW, LR, LL, LSE, LB, LSW of
 *   Fig. restrict_kernel at the coarse point north-east of each F-point triple;
 *   the Galerkin coarse operator P^T A P as a nine-point stencil; and the
 *   square-root-free Cholesky (LDL^T) factor of the coarsest level's matrix
 *   (n_L^2 unknowns in lexicographic order, a band of half-bandwidth n_L + 1,
 *   factored column by column with every sum over increasing index).
 *   stencil: n x n x kind, row-major; kind 5: S, W, O, E, N; kind 9: SW, S, SE,
 *            W, O, E, NW, N, NE (the rows of Fig. stencil_operator, south first).
 *            Signed matrix entries, entries toward boundary vertices zero, the
 *            operator symmetric (A_E(i,j) = A_W(i+1,j) etc. to 1e-14 relative),
 *            A_O > 0, all finite.  Copied; not referenced after the call.
 *   workspace: device buffer of ws_bytes >= bmg_workspace_bytes(); it must
 *            outlive the handle.
 * Synchronises `stream` once (to read the validation and breakdown flags).
 * Errors: BMG_EINVAL (size, kind, NULL, stencil values), BMG_EWORKSPACE,
 * BMG_EBREAKDOWN, BMG_EDEVICE.  *out is NULL on failure. */
bmg_status bmg_setup(bmg_solver **out, const double *stencil, int n, int kind,
                     const bmg_options *o, void *workspace, size_t ws_bytes,
                     bmg_stream stream);

/* One V(nu1,nu2)-cycle (Fig. vcycle_flowchart) on A x = rhs, in the
 * precision of the options (FP32_IR: one refinement step).
 *   rhs, x: n x n row-major; x is the initial guess in and the iterate out.
 *   rel_res: host, nullable; if given, receives ||rhs - A x||_2/||rhs||_2 of
 *   the new iterate (this synchronises the stream).  */
bmg_status bmg_vcycle(bmg_solver *h, const double *rhs, double *x, double *rel_res);

/* Cycles from the initial guess x until ||rhs - A x||_2 / ||rhs||_2 <= tol
 * (checked after every cycle, with a residual computed by error-free
 * transformations, as accurate as one in twice FP64) or max_cycles.
 * FP64: V(nu1,nu2)-cycles on x; once the residual is <= refine_factor * tol,
 * x is carried as the double-FP64 pair x + x_lo and a cycle is one refinement
 * step: r = rhs - A (x + x_lo) (accurate, rounded once), d = V(0, r),
 * (x, x_lo) += d in double-FP64.  FP32_IR: the same refinement from the first
 * step, with d = s V32(0, fl32(r / s)), s the power of two >= ||r||_inf.
 * The residual reported is that of the pair; x receives the high part and
 * BMG_F_XLO the low part.  rhs, x as in bmg_vcycle.
 * info (host, nullable) receives the count, final residual and history.
 * ||rhs|| = 0 gives x = 0 after 0 cycles.  Returns BMG_ENOCONV if max_cycles
 * was reached (x and info still valid), BMG_EDIVERGED if the residual became
 * non-finite or grew 1e3-fold over its initial value. */
bmg_status bmg_solve(bmg_solver *h, const double *rhs, double *x, double tol,
                     bmg_info *info);

/* Releases the handle (host memory only; the workspace stays the caller's). */
bmg_status bmg_destroy(bmg_solver *h);

/* For callers that cannot allocate (code that must not call hipMalloc or any
 * allocating routine: allocation-free serving loops, harnesses that forbid
 * it): bmg_setup followed by bmg_solve and the handle's release, in one call
 * that allocates nothing, neither device nor host memory.  The hierarchy lives
 * in a device array the library owns, BMG_NOALLOC_BYTES per GPU, held by each
 * GPU the library runs on until the process ends; the handle lives on the
 * host stack.  Arguments and results as bmg_setup (stencil, n, kind, options,
 * stream) and bmg_solve (rhs, x, tol, info); the current device must be the
 * one the pointers and the stream belong to.  A problem whose workspace
 * (bmg_workspace_bytes) exceeds BMG_NOALLOC_BYTES is rejected with
 * BMG_EWORKSPACE before any launch (64 MiB: n <= 511 in FP64 and in
 * BMG_FP32_IR).  Every call on one GPU shares that GPU's array, which keeps
 * the last call's contents (the set-up clears what must start at zero):
 * calls that overlap on one GPU, from several threads or streams, race. */
#define BMG_NOALLOC_BYTES ((size_t)64 << 20)
bmg_status bmg_solve_noalloc(const double *stencil, int n, int kind, const bmg_options *o,
                             const double *rhs, double *x, double tol, bmg_info *info,
                             bmg_stream stream);

/* ------------------------------------------------------------------------
 * Block solves: k right-hand sides on one hierarchy.  The solver is bandwidth
 * bound and more data reuse and block solves are the further work Sec. 5
 * names; here every fused pass runs the tiles of all k right-hand sides in one
 * launch, the k workgroups of a tile side by side on one XCD, so the operator
 * and weight rows they share are read from HBM about once for all of them.
 * Each right-hand side follows its own bmg_solve exactly (the same cycles, the
 * same switch to refinement at refine_factor * tol, the same stop rule), so
 * its iterate, history and cycle count are the ones bmg_solve gives it alone.
 * The hierarchy must be FP64 (precision BMG_FP64) with the fused kernels,
 * 1 <= nu1 <= 3 and 1 <= nu2 <= 2.
 * ---------------------------------------------------------------------- */
typedef struct bmg_block bmg_block;

/* Device workspace of a block of k >= 1 right-hand sides on h: per level
 * 3k iterate/right-hand-side arrays, 3k fine-level refinement arrays, and
 * per right-hand side its norm partials, scalars, history and stop flag.
 * Errors: BMG_EINVAL (NULL, k < 1, a hierarchy the block cannot run). */
bmg_status bmg_block_workspace_bytes(const bmg_solver *h, int k, size_t *bytes);

/* A block of k right-hand sides on the hierarchy of h (which must outlive it;
 * the block runs on h's stream and only reads h's operators, weights and
 * coarsest factor).  workspace: device, >= bmg_block_workspace_bytes, owned
 * by the caller, outliving the block.  Errors: BMG_EINVAL, BMG_EWORKSPACE. */
bmg_status bmg_block_create(bmg_block **out, bmg_solver *h, int k, void *workspace, size_t bytes);

/* bmg_solve for the k right-hand sides at once.
 *   rhs: device, k planes of n x n (row-major, plane j = right-hand side j);
 *   x:   device, the same layout: initial guesses in, solutions out;
 *   info: host, k entries, nullable (each entry's history as in bmg_solve);
 *   status: host, k entries, nullable: each right-hand side's bmg_solve status.
 * Returns BMG_OK if every right-hand side converged, else the first failing
 * one's status (all x and info entries still valid). */
bmg_status bmg_block_solve(bmg_block *b, const double *rhs, double *x, double tol, bmg_info *info,
                           bmg_status *status);

/* Kernel timing of the block's fused passes, as bmg_trace_enable/read (the
 * bytes count the operator and weights once and the per-right-hand-side
 * arrays k times). */
bmg_status bmg_block_trace_enable(bmg_block *b, int kclass, int level, int on);
bmg_status bmg_block_trace_read(bmg_block *b, int *launches, double *total_ms, double *bytes);

/* Releases the block (host memory only). */
bmg_status bmg_block_destroy(bmg_block *b);

const char *bmg_status_string(int status);
const char *bmg_last_error(void);

/* ------------------------------------------------------------------------
 * Level access and single steps, on the hierarchy's own level arrays.  These
 * expose each step of the cycle for testing and tracing.
 * ---------------------------------------------------------------------- */

/* Fields of a level.  Transfers use the tight layout:
 *   level arrays: (n_l+2) x (n_l+2) row-major with the Dirichlet ring;
 *   BMG_F_CI: 8 x (n_{l+1}+2) x (n_{l+1}+2), planes LNE, LA, LNW, LR, LL, LSE,
 *   LB, LSW (the weights between level l and l+1);
 *   BMG_F_COARSE_LD: the coarsest factor, m = n_L^2 unknowns, w = n_L + 1:
 *   m x w entries of L in band storage (row i holds L_ik for k = i-w .. i-1
 *   at column k - i + w, zero for k < 0; the unit diagonal is implicit)
 *   followed by the m entries of D (level argument ignored);
 *   BMG_F_XLO: the low part of the last solve's double-FP64 iterate, level-0
 *   layout (zero if the solve never switched to refinement);
 *   BMG_F_STENCIL (export only): the level's operator as bmg_setup reads it,
 *   n_l x n_l x K with K = 5 (S, W, O, E, N) on a five-point level and K = 9
 *   (SW, S, SE, W, O, E, NW, N, NE) otherwise.
 * The *32 fields are the FP32 hierarchy (precision BMG_FP32_IR only) and
 * transfer float data.  A solve or V-cycle leaves the level-0 u32 unspecified:
 * the fused fine-level pass of a refinement step adds each FP32 correction to
 * the double-FP64 iterate in place of storing it. */
enum {
    BMG_F_U = 0, BMG_F_B = 1, BMG_F_R = 2,
    BMG_F_AO = 3, BMG_F_AW = 4, BMG_F_AS = 5, BMG_F_ASW = 6, BMG_F_ANW = 7,
    BMG_F_CI = 8, BMG_F_COARSE_LD = 9, BMG_F_XLO = 10, BMG_F_STENCIL = 11,
    BMG_F_U32 = 16, BMG_F_B32 = 17, BMG_F_R32 = 18,
    BMG_F_AO32 = 19, BMG_F_AW32 = 20, BMG_F_AS32 = 21, BMG_F_ASW32 = 22,
    BMG_F_ANW32 = 23, BMG_F_CI32 = 24
};

bmg_status bmg_num_levels(const bmg_solver *h, int *nlev);
bmg_status bmg_level_n(const bmg_solver *h, int level, int *n);
/* Device-to-device copies in the tight layout; enqueued on the stream. */
bmg_status bmg_export(bmg_solver *h, int level, int field, void *dst);
bmg_status bmg_import(bmg_solver *h, int level, int field, const void *src);

/* Steps on level `level` (all on the handle's arrays, in the precision of
 * the field set named by `fp32`: 0 = FP64, 1 = FP32 hierarchy):
 *   BMG_STEP_SMOOTH:   `arg` four-colour Gauss-Seidel sweeps of u with b;
 *   BMG_STEP_RESIDUAL: r = b - A u;
 *   BMG_STEP_RESTRICT: b_{l+1} = P^T r (Fig. restrict_kernel), u_{l+1} = 0;
 *   BMG_STEP_INTERP:   u += P u_{l+1};
 *   BMG_STEP_COARSE:   u = A^{-1} b on the coarsest level (FP64 factor);
 *   BMG_STEP_PRE:      the fused pre-smoothing pass: arg sweeps, residual and
 *                      restriction (results equal to SMOOTH, RESIDUAL,
 *                      RESTRICT in turn, r left unspecified);
 *   BMG_STEP_POST:     the fused post pass: INTERP then arg sweeps.
 * Enqueued on the stream. */
enum {
    BMG_STEP_SMOOTH = 0, BMG_STEP_RESIDUAL = 1, BMG_STEP_RESTRICT = 2,
    BMG_STEP_INTERP = 3, BMG_STEP_COARSE = 4, BMG_STEP_PRE = 5, BMG_STEP_POST = 6
};
bmg_status bmg_step(bmg_solver *h, int level, int step, int arg, int fp32);

/* Kernel timing with HIP events on the handle's stream.  While enabled, every
 * launch of the kernels of class `kclass` on level `level` is bracketed by an
 * event pair (at most 65536 pairs are kept).  bmg_trace_read synchronises the
 * stream and returns the number of launches timed, their total duration in
 * milliseconds and (bytes, may be NULL) their algorithmic HBM bytes: each
 * array the launch needs counted once, read or written, for the variant that
 * ran (a fused pre pass that computes its weights does not count them).  It
 * then clears the record.  Classes: */
enum { BMG_TRACE_SMOOTH = 0, BMG_TRACE_PRE = 1, BMG_TRACE_POST = 2, BMG_TRACE_RESNORM = 3,
       BMG_TRACE_POSTPRE = 4 /* fine post pass fused with the next cycle's fine pre pass */ };
bmg_status bmg_trace_enable(bmg_solver *h, int kclass, int level, int on);
bmg_status bmg_trace_read(bmg_solver *h, int *launches, double *total_ms, double *bytes);

/* ------------------------------------------------------------------------
 * Tile shapes of the fused passes.  A process-wide table of rows per tile for
 * each level size n = 2^m - 1, written by the autotuner; 0 restores the
 * built-in default.  bmg_options.tile_rows, when set, overrides the table.
 * ---------------------------------------------------------------------- */
bmg_status bmg_tile_rows_set(int n, int rows);
bmg_status bmg_tile_rows_get(int n, int *rows);

/* ------------------------------------------------------------------------
 * Batched solves: nprob independent problems of uneven sizes (n[p] = 2^m - 1,
 * n[p] >= 7, five-point operators as for bmg_setup), FP32 V(2,1)-cycles
 * inside double-FP64 iterative refinement (the precision option is ignored),
 * advanced together by one persistent cooperative launch per group of steps
 * that runs every problem's refinement steps phase by phase with a
 * device-side stop flag per problem (a replay from a HIP graph is tried first;
 * where the runtime replays the cooperative node without its grid barrier,
 * direct cooperative launches run it, see bmg_batch_info).  Each problem's iterates equal those of
 * bmg_solve with precision BMG_FP32_IR.
 * ---------------------------------------------------------------------- */
typedef struct bmg_batch bmg_batch;

/* n: host array of nprob sizes.  Host only. */
bmg_status bmg_batch_workspace_bytes(int nprob, const int *n, const bmg_options *o, size_t *bytes);

/* stencils: host array of nprob device pointers, each n[p] x n[p] x 5.
 * Synchronises the stream (once per problem while setting up). */
bmg_status bmg_batch_setup(bmg_batch **out, int nprob, const int *n, const double *const *stencils,
                           const bmg_options *o, void *workspace, size_t ws_bytes, bmg_stream stream);

/* rhs, x: host arrays of nprob device pointers to n[p] x n[p] arrays (x is the
 * initial guess in, the solution's high part out).  steps (host, nullable)
 * receives each problem's refinement steps, rel_res (host, nullable) its final
 * relative residual.  BMG_ENOCONV / BMG_EDIVERGED name the first problem that
 * failed; the others are still solved. */
bmg_status bmg_batch_solve(bmg_batch *h, const double *const *rhs, double *const *x, double tol,
                           int *steps, double *rel_res);

/* Residual history of problem p: hist[0] is the initial relative residual,
 * hist[k] the one after step k; *count entries exist (up to cap copied). */
bmg_status bmg_batch_history(bmg_batch *h, int p, double *hist, int cap, int *count);

/* Workgroups of the persistent launch and how it is launched: graph_used = 1
 * replayed from a HIP graph (one cooperative kernel node); 0 the runtime could
 * not build that graph; 2 a replay ran without the grid barrier (detected by
 * the kernel before any work) and direct cooperative launches took over. */
bmg_status bmg_batch_info(const bmg_batch *h, int *nblocks, int *graph_used);
bmg_status bmg_batch_destroy(bmg_batch *h);

/* ------------------------------------------------------------------------
 * Learned interpolation (an addition; the paper's interpolation is the
 * operator-induced one).  A convolutional network reads the nine stencil
 * coefficients of every fine point, each divided by the centre coefficient,
 * and writes the eight weight planes of the coarse level in the layout of the
 * operator-induced weights (LNE, LA, LNW, LR, LL, LSE, LB, LSW, stored at the
 * north-east coarse point of each F-point triple; weights of F-points that do
 * not exist are zero).  Layers: 3x3 conv 9->32 with ReLU at every fine point;
 * 3x3 conv 32->32, stride 2, with ReLU at the coarse points (I, J),
 * I, J = 1..nc+1, centred on the fine point (2I, 2J); 3x3 conv 32->8, linear,
 * at the same points; zero padding.  Weights and activations are bfloat16
 * (round to nearest even), products accumulate in FP32 on the matrix cores
 * (MFMA), biases are FP32.
 *
 * Parameters are a flat FP32 vector of BMG_NET_PARAMS values: conv1 weights
 * [tap][in 9][out 32], bias [32], conv2 weights [tap][32][32], bias [32],
 * conv3 weights [tap][32][8], bias [8]; tap t = 3 (dy + 1) + (dx + 1) reads
 * the point offset by (dx, dy).
 *
 * Training minimises the two-grid residual reduction ||r3||^2 / ||r0||^2 of
 * one cycle (one GS sweep, coarse correction with A_c = P^T A P solved by
 * V-cycles to a tolerance, one GS sweep) on A x = r0 from x = 0, with the
 * gradient from the adjoint of that cycle and Adam updates.
 * ---------------------------------------------------------------------- */
#define BMG_NET_PARAMS 14184

/* Device workspace of a network used on levels of up to max_n points per side;
 * train = 0 sizes it for inference only (no backward pass or two-grid
 * training).  Host only. */
bmg_status bmg_net_workspace_bytes(int max_n, int train, size_t *bytes);

/* params: host, BMG_NET_PARAMS floats.  Adam moments start at zero.  The
 * handle keeps pointers into the workspace and uses `stream`. */
bmg_status bmg_net_create(bmg_net **out, int max_n, int train, const float *params, void *workspace,
                          size_t ws_bytes, bmg_stream stream);
bmg_status bmg_net_set_params(bmg_net *net, const float *params /* host */);
bmg_status bmg_net_get_params(bmg_net *net, float *params /* host */);
bmg_status bmg_net_destroy(bmg_net *net);

/* Forward pass on one level given by its padded compact planes ((n+2) rows of
 * pitch ld; SW and NW NULL for a five-point level) into the weight planes
 * Ci (8 planes of (nc+2) rows of pitch ldc, plane stride ps, every entry
 * written).  The weights are BoxMG's operator-induced ones plus the network's
 * eight outputs at each coarse point as corrections that keep each F-point's
 * weight sum: x-edge e = (y_LR - y_LL) / 2 added to LR and taken from LL,
 * y-edge likewise with LA, LB, and the corner weights each y_w minus the
 * mean of the four; F-points that do not exist keep zero weights.  A zero
 * network therefore gives BoxMG's weights.  The activations stay in the
 * workspace for bmg_net_backward. */
bmg_status bmg_net_forward(bmg_net *net, int n, int ld, const double *O, const double *W, const double *S,
                           const double *SW, const double *NW, double *Ci, int ldc, size_t ps);

/* Backward pass of the last forward pass (train = 1): given dL/dCi in the
 * layout of bmg_net_forward's output, adds dL/dparams to the gradient sum. */
bmg_status bmg_net_backward(bmg_net *net, const double *dCi, int ldc, size_t ps);

/* The gradient sum (host, BMG_NET_PARAMS doubles); zeroing it. */
bmg_status bmg_net_get_grad(bmg_net *net, double *grad);
bmg_status bmg_net_zero_grad(bmg_net *net);

/* One Adam step (Kingma and Ba) in FP32 with gradient = scale * sum, step
 * counter advanced by one; the bfloat16 weights follow the new parameters. */
bmg_status bmg_net_adam(bmg_net *net, float lr, float beta1, float beta2, float eps, double scale);

/* Intermediate arrays of the last passes, device-to-device, bfloat16 bits in
 * point-major layout (channels innermost):
 *   X  (n+2)^2 x 16 (9 used),  H1 (n+3)^2 x 32,  H2 (nc+3)^2 x 32,
 *   D3 (nc+3)^2 x 16 (8 used), D2 (nc+3)^2 x 32, D1 (n+2)^2 x 32,
 * and the output layer's values Y, (nc+2)^2 x 8 FP32,
 * with point (i, j) at j * (side) + i.  *bytes receives the size. */
enum { BMG_NET_X = 0, BMG_NET_H1 = 1, BMG_NET_H2 = 2, BMG_NET_D3 = 3, BMG_NET_D2 = 4, BMG_NET_D1 = 5,
       BMG_NET_Y = 6 };
bmg_status bmg_net_export(bmg_net *net, int what, void *dst, size_t *bytes);

/* One training sample: h must have been set up with BMG_INTERP_LEARNED,
 * learned_levels = 1 and this network on the level's operator (n >= 7), and
 * nothing run on `net` since.  r0: n x n (device).  Runs the two-grid cycle,
 * its adjoint (coarse solves by V(nu1,nu2)-cycles of h from level 1 until
 * the relative residual is <= inner_tol or inner_max cycles), and the
 * network's backward pass, which adds to the gradient sum.  loss (host)
 * receives ||r3||^2 / ||r0||^2; dCi (device, nullable) a copy of dL/dCi in
 * the layout of the level's weight planes (bmg_export of BMG_F_CI). */
bmg_status bmg_net_twogrid(bmg_net *net, bmg_solver *h, const double *r0, double inner_tol, int inner_max,
                           double *loss, double *dCi);

/* The fallback rule of the learned interpolation: both handles (set up on the
 * same operator, `learned` with BMG_INTERP_LEARNED, `boxmg` with the
 * operator-induced weights) run probe_cycles V-cycles (0 = 8) from x; the
 * measured reduction factor of each is the mean per cycle over the second
 * half of its probe, rho = (r_K / r_(K/2))^(2/K) with K = probe_cycles, and
 * the hierarchy with the smaller one (the learned one on a tie) continues
 * from its own iterate with bmg_solve.  The learned hierarchy is watched: it
 * runs in chunks of 16 cycles, and a chunk whose mean factor exceeds the BoxMG
 * probe's hands the current iterate (still valid) to the BoxMG hierarchy for
 * the rest of the solve.  used (host) receives the hierarchy that finished,
 * BMG_INTERP_LEARNED or BMG_INTERP_BOXMG; rho (host, 2 entries) the probe
 * factors of the learned and the BoxMG hierarchy; info->cycles counts every
 * cycle after the probes plus the finishing hierarchy's probe, the other
 * fields describe the last bmg_solve call, except info->history (if given,
 * max_cycles + 1 entries), which receives the relative residual after each
 * cycle that followed the probes, in order, and info->interp_used, the
 * hierarchy that finished.  FP64 handles only. */
bmg_status bmg_solve_select(bmg_solver *learned, bmg_solver *boxmg, const double *rhs, double *x, double tol,
                            int probe_cycles, bmg_info *info, int *used, double *rho);

/* ------------------------------------------------------------------------
 * Nonsymmetric black-box multigrid (operators with A != A^T, e.g.
 * convection-diffusion): the member of the BoxMG family the paper's
 * references (Section 1) describe for nonsymmetric problems, with the V-cycle
 * of Fig. vcycle_flowchart.  Interpolation P is induced by A with the
 * symmetric solver's collapse formulas; the restriction is R = P~^T, P~ the
 * interpolation the same formulas induce from A^T, applied with the term
 * order of Fig. restrict_kernel; the coarse operators are R A P in all nine
 * directions; every level stores all nine entries of each row; relaxation is
 * four-colour Gauss-Seidel (one launch per colour); the coarsest level (size
 * coarsest_n, 3 by default, at most 63) is factored as a band L D U (unit
 * triangular L and U) and solved by the one-wave band substitutions, each
 * update one fused multiply-add.  Options used: nu1, nu2, max_cycles,
 * coarsest_n; precision, smoother and interpolation must be the defaults.
 * ---------------------------------------------------------------------- */
typedef struct bmg_ns bmg_ns;

/* Device workspace of a nonsymmetric hierarchy (host only). */
bmg_status bmg_ns_workspace_bytes(int n, int kind, const bmg_options *o, size_t *bytes);

/* Set-up from the stencil (device, [n][n][K], K = 5: S, W, O, E, N; K = 9: SW,
 * S, SE, W, O, E, NW, N, NE; signed matrix entries, entries toward boundary
 * vertices zero, no symmetry required).  Ownership, alignment and errors as
 * bmg_setup; BMG_EBREAKDOWN if an interpolation denominator or a pivot of the
 * coarsest factor is not positive. */
bmg_status bmg_ns_setup(bmg_ns **out, const double *stencil, int n, int kind, const bmg_options *o,
                        void *workspace, size_t ws_bytes, bmg_stream stream);

/* V(nu1,nu2)-cycles from the initial guess x (device, n x n, in/out) until
 * ||rhs - A x||_2 / ||rhs||_2 <= tol (plain FP64 residual, checked after every
 * cycle) or max_cycles.  info (host, nullable): cycles, final residual, mean
 * factor and, if info->history is given (max_cycles entries), the residual
 * after each cycle.  BMG_ENOCONV / BMG_EDIVERGED as bmg_solve; ||rhs|| = 0
 * gives x = 0 after 0 cycles. */
bmg_status bmg_ns_solve(bmg_ns *h, const double *rhs, double *x, double tol, bmg_info *info);
bmg_status bmg_ns_destroy(bmg_ns *h);

/* Level access for tests: fields 0..8 the stencil planes (SW..NE), 9 P's and
 * 10 R's weights (8 planes of the coarse level's (nc+2)^2 shape), 11 u, 12 b,
 * 13 r (padded (n+2)^2, tight on output), 14 the coarsest factor (L band
 * m x w, U band m x w with U_ik at i w + (k - i - 1), D m).  Import takes u, b,
 * r.  Steps: 0 = arg sweeps, 1 = residual, 2 = restriction of r into the next
 * level's b (its u zeroed), 3 = u += P u_next, 4 = the coarsest solve.  All
 * synchronous on the handle's stream. */
bmg_status bmg_ns_num_levels(const bmg_ns *h, int *nlev);
bmg_status bmg_ns_level_n(const bmg_ns *h, int level, int *n);
bmg_status bmg_ns_export(bmg_ns *h, int level, int field, double *dst);
bmg_status bmg_ns_import(bmg_ns *h, int level, int field, const double *src);
bmg_status bmg_ns_step(bmg_ns *h, int level, int step, int arg);

#ifdef __cplusplus
}
#endif

#endif /* BMG_H */
