// Batched solves: many independent problems of uneven sizes, FP32 V-cycles
// inside double-FP64 iterative refinement, all advanced by one persistent,
// cooperative launch.
//
// Each problem keeps its own hierarchy (set up by the single-problem path in
// its own slice of the workspace).  The persistent kernel walks a fixed list
// of phases per refinement step; every phase is a list of work items (row
// chunks of a problem's fine grid, tiles of one level of a problem, or whole
// problems) dealt round-robin to the resident workgroups, and phases are
// separated by grid-wide barriers:
//   OUTER   r = b - A (x_hi + x_lo) in FP64 (accurate), partial ||r||^2, max|r|
//   DECIDE  per problem: record ||r||/||b||, stop test, power-of-two scale s
//   SCALE   b32 = fl32(r / s), u32 = 0
//   PRE(d)  fused pre pass of every problem's level d (d = 0, 1, ...)
//   SMALL   the sub-cycle of every problem's levels of at most 63 points
//   POST(d) fused post pass, d descending
//   UPDATE  (x_hi, x_lo) += s u32
// Problems that have stopped skip their items; a step in which every problem
// has stopped ends the launch.  Each problem's iterates are those of the
// single-problem solver, bit for bit.
#include "bmg_internal.hpp"

#include <hip/hip_cooperative_groups.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

using namespace bmgi;
namespace cg = cooperative_groups;

namespace {

constexpr int BT = FW;              // threads per workgroup (one fused tile)
constexpr int CHUNK_ROWS = 16;      // fine rows per item of the FP64 phases
constexpr int MAXD = 8;             // tiled levels per problem (n > SMALL_BATCH)
// Levels of at most this many points per side run in the per-problem
// LDS-resident sub-cycle.  31 keeps the kernel's LDS at the size of one
// nine-point FP32 tile (four workgroups per CU); 63 runs one more level per
// problem in LDS (two workgroups per CU, two fewer grid barriers per step).
#ifndef BMG_BATCH_SMALL_N
#define BMG_BATCH_SMALL_N 31
#endif
constexpr int SMALL_BATCH = BMG_BATCH_SMALL_N;

struct BProb {
    int n0, nlev, sdepth;           // finest size, levels, first small level
    int nchunks;
    Lev<float> L[MAXL];             // FP32 hierarchy, u = the level's input buffer
    Wts<float> C[MAXL];
    float *ualt[MAXL];              // second iterate buffer of each level
    TileGeo gpre[MAXD], gpost[MAXD];
    SmallH<float> small;
    Lev<double> L0;                 // FP64 fine level: stencil and r
    double *B0, *XH, *XL;
    double *part;                   // per chunk: sum of squares, max |r|
    double *hist;                   // relative residual per refinement step
    const double *rhs;              // caller's arrays, n0 x n0
    double *x;
    double bnorm, rel0, scale;
    int count, done;                // history entries; stop code (0 running)
};

struct BLists {
    int chunk0, chunk1, prob0, prob1;
    int pre0[MAXD], pre1[MAXD], post0[MAXD], post1[MAXD];
    int ndepth;
};

struct BArgs {
    BProb *P;
    const int2 *items;
    BLists li;
    int nprob;
    double tol;
    int maxc;
    int *active;                    // problems still running after the launch
};

__device__ __forceinline__ double block_max(double v)
{
    __shared__ double part[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (wid == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        v = lane < nw ? part[lane] : 0.0;
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    }
    return v;
}

// Accurate FP64 residual of the five-point fine level, as k_resid_dd.
__device__ __forceinline__ double fine_residual(const BProb &q, size_t p)
{
    const Lev<double> &L = q.L0;
    const size_t ld = L.ld;
    const size_t qq[5] = {p - ld, p - 1, p + 1, p + ld, p};
    const double a[5] = {L.S[p], L.W[p], L.W[p + 1], L.S[p + ld], L.O[p]};
    double s = q.B0[p], c = 0.0, ns, se;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const double x = q.XH[qq[t]];
        const double pr = a[t] * x;
        const double pe = fma(a[t], x, -pr);
        two_sum(s, -pr, ns, se);
        s = ns;
        c = c + (se - pe);
    }
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        two_sum(s, -(a[t] * q.XL[qq[t]]), ns, se);
        s = ns;
        c = c + se;
    }
    return s + c;
}

enum { MODE_INIT = 1, MODE_STEPS = 2, MODE_FINISH = 3 };

// Grid-wide barrier followed by a device-scope fence, so that every load after
// it (through this CU's L1 and this XCD's L2) sees what other workgroups wrote
// before the barrier.
__device__ __forceinline__ void phase_barrier(cg::grid_group &grid)
{
    grid.sync();
    __threadfence();
}

__global__ __launch_bounds__(BT, 4) void k_batch(BArgs A, int mode, int steps)
{
    extern __shared__ unsigned char smem[];
    cg::grid_group grid = cg::this_grid();
    BProb *P = A.P;
    const int2 *items = A.items;
    const int nb = gridDim.x, bid = blockIdx.x;
    // a launch that is not cooperative has no grid barrier: leave at once,
    // before any barrier, and tell the host through the active count
    if (!grid.is_valid()) {
        if (bid == 0 && threadIdx.x == 0) *A.active = -1;
        return;
    }

    if (mode == MODE_INIT) {
        // pack the caller's arrays, x_lo = 0, and ||b||^2 by chunks
        for (int it = A.li.chunk0 + bid; it < A.li.chunk1; it += nb) {
            BProb &q = P[items[it].x];
            const int c = items[it].y, n = q.n0, ld = q.L0.ld;
            const int j0 = 1 + c * CHUNK_ROWS, j1 = min(n, j0 + CHUNK_ROWS - 1);
            double acc = 0.0;
            for (int j = j0; j <= j1; ++j)
                for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x) {
                    const size_t p = (size_t)j * ld + i, s = (size_t)(j - 1) * n + (i - 1);
                    const double b = q.rhs[s];
                    q.B0[p] = b;
                    q.XH[p] = q.x[s];
                    q.XL[p] = 0.0;
                    acc += b * b;
                }
            acc = block_sum(acc);
            if (threadIdx.x == 0) q.part[2 * c] = acc;
            __syncthreads();
        }
        phase_barrier(grid);
        for (int it = A.li.prob0 + bid; it < A.li.prob1; it += nb) {
            BProb &q = P[items[it].x];
            if (threadIdx.x == 0) {
                double s = 0.0;
                for (int c = 0; c < q.nchunks; ++c) s += q.part[2 * c];
                q.bnorm = sqrt(s);
                q.count = 0;
                q.done = s == 0.0 ? 5 : 0;   // zero right-hand side: x = 0, no steps
            }
        }
        return;
    }
    if (mode == MODE_FINISH) {
        for (int it = A.li.chunk0 + bid; it < A.li.chunk1; it += nb) {
            BProb &q = P[items[it].x];
            const int c = items[it].y, n = q.n0, ld = q.L0.ld;
            const int j0 = 1 + c * CHUNK_ROWS, j1 = min(n, j0 + CHUNK_ROWS - 1);
            const bool zero = q.done == 5;
            for (int j = j0; j <= j1; ++j)
                for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x)
                    q.x[(size_t)(j - 1) * n + (i - 1)] = zero ? 0.0 : q.XH[(size_t)j * ld + i];
        }
        return;
    }

    for (int step = 0; step < steps; ++step) {
        // OUTER: accurate FP64 residual of the pair, by row chunks
        for (int it = A.li.chunk0 + bid; it < A.li.chunk1; it += nb) {
            BProb &q = P[items[it].x];
            if (q.done) continue;
            const int c = items[it].y, n = q.n0, ld = q.L0.ld;
            const int j0 = 1 + c * CHUNK_ROWS, j1 = min(n, j0 + CHUNK_ROWS - 1);
            double acc = 0.0, mx = 0.0;
            for (int j = j0; j <= j1; ++j)
                for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x) {
                    const size_t p = (size_t)j * ld + i;
                    const double r = fine_residual(q, p);
                    q.L0.r[p] = r;
                    acc += r * r;
                    mx = fmax(mx, fabs(r));
                }
            acc = block_sum(acc);
            __syncthreads();
            mx = block_max(mx);
            if (threadIdx.x == 0) {
                q.part[2 * c] = acc;
                q.part[2 * c + 1] = mx;
            }
            __syncthreads();
        }
        phase_barrier(grid);
        // DECIDE: history, stop test, scale (one thread per problem)
        for (int it = A.li.prob0 + bid; it < A.li.prob1; it += nb) {
            BProb &q = P[items[it].x];
            if (threadIdx.x != 0 || q.done) continue;
            double s = 0.0, mx = 0.0;
            for (int c = 0; c < q.nchunks; ++c) {
                s += q.part[2 * c];
                mx = fmax(mx, q.part[2 * c + 1]);
            }
            const double rel = sqrt(s) / q.bnorm;
            const int k = q.count;
            q.hist[k] = rel;
            if (k == 0) q.rel0 = rel;
            q.count = k + 1;
            if (rel <= A.tol) q.done = 1;
            else if (!isfinite(rel) || rel > 1e3 * q.rel0) q.done = 2;
            else if (k + 1 >= A.maxc) q.done = 3;
            else {
                int e = 0;
                const double fr = frexp(mx, &e);
                if (fr == 0.5) e -= 1;
                if (fr == 0.0) e = 0;
                q.scale = ldexp(1.0, e);
            }
        }
        phase_barrier(grid);
        {
            int running = 0;
            for (int p = 0; p < A.nprob; ++p) running += P[p].done == 0;
            if (running == 0) {
                if (bid == 0 && threadIdx.x == 0) *A.active = 0;
                return;
            }
        }
        // SCALE: b32 = fl32(r / s), u32 = 0
        for (int it = A.li.chunk0 + bid; it < A.li.chunk1; it += nb) {
            BProb &q = P[items[it].x];
            if (q.done) continue;
            const int c = items[it].y, n = q.n0, ld = q.L0.ld;
            const int j0 = 1 + c * CHUNK_ROWS, j1 = min(n, j0 + CHUNK_ROWS - 1);
            const double inv = 1.0 / q.scale;       // exact: a power of two
            for (int j = j0; j <= j1; ++j)
                for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x) {
                    const size_t p = (size_t)j * ld + i;
                    q.L[0].b[p] = (float)(q.L0.r[p] * inv);
                    q.L[0].u[p] = 0.0f;
                }
        }
        phase_barrier(grid);
        // PRE(d): fused nu1 = 2 sweeps, residual, restriction, by tiles
        for (int d = 0; d < A.li.ndepth; ++d) {
            for (int it = A.li.pre0[d] + bid; it < A.li.pre1[d]; it += nb) {
                BProb &q = P[items[it].x];
                if (q.done) continue;
                if (d == 0)
                    pre_tile<float, false, 2>(q.L[0], q.ualt[0], q.C[0], q.L[1], q.gpre[0], items[it].y,
                                              *reinterpret_cast<TileLds<float, false, 2> *>(smem));
                else
                    pre_tile<float, true, 2>(q.L[d], q.ualt[d], q.C[d], q.L[d + 1], q.gpre[d], items[it].y,
                                             *reinterpret_cast<TileLds<float, true, 2> *>(smem));
                __syncthreads();
            }
            phase_barrier(grid);
        }
        // SMALL: the sub-cycle of the levels of at most 63 points, per problem
        for (int it = A.li.prob0 + bid; it < A.li.prob1; it += nb) {
            BProb &q = P[items[it].x];
            if (q.done) continue;
            if (q.sdepth == 0) small_vcycle_body<float, false>(q.small, reinterpret_cast<float *>(smem), 0);
            else small_vcycle_body<float, true>(q.small, reinterpret_cast<float *>(smem), 0);
            __syncthreads();
        }
        phase_barrier(grid);
        // POST(d): interpolation and nu2 = 1 sweep, d descending
        for (int d = A.li.ndepth - 1; d >= 0; --d) {
            for (int it = A.li.post0[d] + bid; it < A.li.post1[d]; it += nb) {
                BProb &q = P[items[it].x];
                if (q.done) continue;
                Lev<float> L = q.L[d];
                float *out = L.u;
                L.u = q.ualt[d];
                if (d == 0)
                    post_tile<float, false, 1, false>(L, out, q.C[0], q.L[1].u, q.gpost[0], items[it].y, nullptr,
                                                      *reinterpret_cast<TileLds<float, false, 1> *>(smem));
                else
                    post_tile<float, true, 1, false>(L, out, q.C[d], q.L[d + 1].u, q.gpost[d], items[it].y, nullptr,
                                                     *reinterpret_cast<TileLds<float, true, 1> *>(smem));
                __syncthreads();
            }
            phase_barrier(grid);
        }
        // UPDATE: (x_hi, x_lo) += s u32
        for (int it = A.li.chunk0 + bid; it < A.li.chunk1; it += nb) {
            BProb &q = P[items[it].x];
            if (q.done) continue;
            const int c = items[it].y, n = q.n0, ld = q.L0.ld;
            const int j0 = 1 + c * CHUNK_ROWS, j1 = min(n, j0 + CHUNK_ROWS - 1);
            for (int j = j0; j <= j1; ++j)
                for (int i = 1 + threadIdx.x; i <= n; i += blockDim.x) {
                    const size_t p = (size_t)j * ld + i;
                    const double dd = q.scale * (double)q.L[0].u[p];
                    double s, e;
                    two_sum(q.XH[p], dd, s, e);
                    e = e + q.XL[p];
                    const double hi = s + e;
                    q.XL[p] = e - (hi - s);
                    q.XH[p] = hi;
                }
        }
        phase_barrier(grid);
    }
    if (bid == 0 && threadIdx.x == 0) {
        int running = 0;
        for (int p = 0; p < A.nprob; ++p) running += P[p].done == 0;
        *A.active = running;
    }
}

size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

// Work items of one problem of size n, an upper bound for any tile height:
// row chunks of the FP64 phases (three lists), one item per problem in two
// lists, and the pre and post tiles of every tiled level with two-row tiles
// and the widest halo (nine-point, nu = 2).
size_t max_items(int n)
{
    const size_t nch = (n + CHUNK_ROWS - 1) / CHUNK_ROWS;
    size_t t = 3 * nch + 2;
    const int useful = FW - 2 * (4 * 2 + 2);
    for (int m = n; m > SMALL_BATCH; m = (m - 1) / 2)
        t += 2 * (size_t)((m + useful - 1) / useful) * (size_t)((m + 1) / 2);
    return t;
}

}  // namespace

struct bmg_batch {
    int nprob = 0;
    hipStream_t st = nullptr;
    std::vector<bmg_solver *> sub;
    std::vector<int> n;
    BProb *dP = nullptr;
    int2 *ditems = nullptr;
    int *dactive = nullptr;
    BLists li{};
    int nitems = 0;
    int maxc = 0;
    int nblocks = 0;
    size_t lds = 0;
    bool graph_tried = false, graph_ok = false;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    bool graph_refused = false;     // a replay ran without the grid barrier
    int graph_steps = 0;
    double graph_tol = -1.0;
};

namespace {

bmg_options batch_options(const bmg_options *o)
{
    bmg_options op;
    bmg_default_options(&op);
    if (o) op = *o;
    op.precision = BMG_FP32_IR;
    op.kernels = BMG_KERNELS_FUSED;
    return op;
}

// Workspace of the batch: the problems' slices, then the problem table, the
// item list and the per-problem partial sums and histories.
size_t batch_layout(int nprob, const int *n, const bmg_options &op, std::vector<size_t> *offs,
                    size_t *tail)
{
    size_t off = 0;
    for (int p = 0; p < nprob; ++p) {
        size_t b = 0;
        if (bmg_workspace_bytes(n[p], 5, &op, &b) != BMG_OK) return 0;
        if (offs) offs->push_back(off);
        off = align_up(off + b);
    }
    if (tail) *tail = off;
    size_t items = 0, parts = 0;
    for (int p = 0; p < nprob; ++p) {
        const int nch = (n[p] + CHUNK_ROWS - 1) / CHUNK_ROWS;
        items += max_items(n[p]);
        parts += 2 * (size_t)nch;
    }
    off = align_up(off + (size_t)nprob * sizeof(BProb));
    off = align_up(off + items * sizeof(int2));
    off = align_up(off + parts * sizeof(double));
    off = align_up(off + (size_t)nprob * (op.max_cycles + 2) * sizeof(double));
    off = align_up(off + 64);
    return off;
}

}  // namespace

extern "C" {

bmg_status bmg_batch_workspace_bytes(int nprob, const int *n, const bmg_options *o, size_t *bytes)
{
    if (nprob < 1 || !n || !bytes) return fail(BMG_EINVAL, "bad batch arguments");
    for (int p = 0; p < nprob; ++p)
        if (!valid_n(n[p]) || n[p] < 7) return fail(BMG_EINVAL, "problem %d: n=%d is not 2^m-1 >= 7", p, n[p]);
    const bmg_options op = batch_options(o);
    if (op.nu1 != 2 || op.nu2 != 1) return fail(BMG_EINVAL, "the batched path runs V(2,1) cycles");
    if (op.coarsest_n != 0 && op.coarsest_n != 3)
        return fail(BMG_EINVAL, "the batched path solves a 3 x 3 coarsest level (coarsest_n = %d)", op.coarsest_n);
    *bytes = batch_layout(nprob, n, op, nullptr, nullptr);
    return *bytes ? BMG_OK : fail(BMG_EINVAL, "bad batch options");
}

bmg_status bmg_batch_setup(bmg_batch **out, int nprob, const int *n, const double *const *stencils,
                           const bmg_options *o, void *workspace, size_t ws_bytes, bmg_stream stream)
{
    if (!out) return fail(BMG_EINVAL, "out pointer is NULL");
    *out = nullptr;
    size_t need = 0;
    TRY(bmg_batch_workspace_bytes(nprob, n, o, &need));
    if (!stencils) return fail(BMG_EINVAL, "stencils is NULL");
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace & (ALIGN - 1)))
        return fail(BMG_EWORKSPACE, "workspace of %zu bytes; need %zu, 256-byte aligned", ws_bytes, need);
    const bmg_options op = batch_options(o);
    std::vector<size_t> offs;
    size_t tail = 0;
    batch_layout(nprob, n, op, &offs, &tail);
    bmg_batch *B = new bmg_batch();
    B->nprob = nprob;
    B->st = (hipStream_t)stream;
    B->n.assign(n, n + nprob);
    B->maxc = op.max_cycles + 1;
    auto bail = [&](bmg_status s) {
        for (bmg_solver *h : B->sub) bmg_destroy(h);
        delete B;
        return s;
    };
    char *ws = (char *)workspace;
    for (int p = 0; p < nprob; ++p) {
        bmg_solver *h = nullptr;
        size_t b = 0;
        bmg_workspace_bytes(n[p], 5, &op, &b);
        const bmg_status s = bmg_setup(&h, stencils[p], n[p], 5, &op, ws + offs[p], b, stream);
        if (s != BMG_OK) return bail(fail(s, "problem %d: %s", p, bmg_last_error()));
        B->sub.push_back(h);
    }
    // problem table, work items
    size_t off = tail;
    B->dP = (BProb *)(ws + off);
    off = align_up(off + (size_t)nprob * sizeof(BProb));
    B->ditems = (int2 *)(ws + off);
    size_t items_cap = 0, parts = 0;
    for (int p = 0; p < nprob; ++p) {
        const int nch = (n[p] + CHUNK_ROWS - 1) / CHUNK_ROWS;
        items_cap += max_items(n[p]);
        parts += 2 * (size_t)nch;
    }
    off = align_up(off + items_cap * sizeof(int2));
    double *dpart = (double *)(ws + off);
    off = align_up(off + parts * sizeof(double));
    double *dhist = (double *)(ws + off);
    off = align_up(off + (size_t)nprob * (op.max_cycles + 2) * sizeof(double));
    B->dactive = (int *)(ws + off);

    std::vector<BProb> hp(nprob);
    std::vector<int2> chunks, probs, pre[MAXD], post[MAXD];
    size_t part_off = 0;
    int ndepth = 0;
    for (int p = 0; p < nprob; ++p) {
        bmg_solver *h = B->sub[p];
        BProb &q = hp[p];
        memset(&q, 0, sizeof q);
        q.n0 = n[p];
        q.nlev = h->nlev;
        q.sdepth = 0;
        while (q.sdepth < h->nlev - 1 && h->L32[q.sdepth].n > SMALL_BATCH) ++q.sdepth;
        if (q.sdepth > MAXD) return bail(fail(BMG_EINVAL, "problem %d is too large for the batch", p));
        ndepth = std::max(ndepth, q.sdepth);
        for (int l = 0; l < h->nlev; ++l) {
            q.L[l] = h->L32[l];
            q.C[l] = h->C32[l];
            q.ualt[l] = h->ualt32[l];
        }
        for (int d = 0; d < q.sdepth; ++d) {
            const int nl = h->L32[d].n, rows = tile_rows_for(h, nl, h->nine[d]);
            q.gpre[d] = tile_geo(nl, d == 0 ? 6 : 10, rows);
            q.gpost[d] = tile_geo(nl, d == 0 ? 4 : 6, rows);
            for (int t = 0; t < q.gpre[d].ntiles; ++t) pre[d].push_back(make_int2(p, t));
            for (int t = 0; t < q.gpost[d].ntiles; ++t) post[d].push_back(make_int2(p, t));
        }
        SmallH<float> &S = q.small;
        S.nl = h->nlev - q.sdepth;
        if (S.nl > SMALL_MAXL) return bail(fail(BMG_EINVAL, "problem %d: too many small levels", p));
        for (int k = 0; k < S.nl; ++k) {
            S.L[k] = h->L32[q.sdepth + k];
            if (k + 1 < S.nl) S.C[k] = h->C32[q.sdepth + k];
        }
        const int lds_small = small_layout(S) * (int)sizeof(float);
        B->lds = std::max(B->lds, (size_t)lds_small);
        S.band = h->band;
        S.nu1 = 2;
        S.nu2 = 1;
        q.L0 = h->L[0];
        q.B0 = h->B0;
        q.XH = h->XH;
        q.XL = h->XL;
        q.nchunks = (n[p] + CHUNK_ROWS - 1) / CHUNK_ROWS;
        q.part = dpart + part_off;
        part_off += 2 * (size_t)q.nchunks;
        q.hist = dhist + (size_t)p * (op.max_cycles + 2);
        for (int c = 0; c < q.nchunks; ++c) chunks.push_back(make_int2(p, c));
        probs.push_back(make_int2(p, 0));
    }
    // big problems first inside every list, so the tail of a phase is short
    std::vector<int2> all;
    auto put = [&](std::vector<int2> &v, int &a, int &b) {
        std::stable_sort(v.begin(), v.end(), [&](int2 x, int2 y) { return n[x.x] > n[y.x]; });
        a = (int)all.size();
        all.insert(all.end(), v.begin(), v.end());
        b = (int)all.size();
    };
    put(chunks, B->li.chunk0, B->li.chunk1);
    put(probs, B->li.prob0, B->li.prob1);
    for (int d = 0; d < MAXD; ++d) {
        put(pre[d], B->li.pre0[d], B->li.pre1[d]);
        put(post[d], B->li.post0[d], B->li.post1[d]);
    }
    B->li.ndepth = ndepth;
    if (all.size() > items_cap) return bail(fail(BMG_EINVAL, "item list overflow"));
    B->nitems = (int)all.size();
    B->lds = std::max({B->lds, sizeof(TileLds<float, true, 2>), sizeof(TileLds<float, false, 2>),
                       sizeof(TileLds<float, true, 1>)});
    if (hipMemcpyAsync(B->dP, hp.data(), hp.size() * sizeof(BProb), hipMemcpyHostToDevice, B->st) != hipSuccess ||
        hipMemcpyAsync(B->ditems, all.data(), all.size() * sizeof(int2), hipMemcpyHostToDevice, B->st) != hipSuccess ||
        hipStreamSynchronize(B->st) != hipSuccess)
        return bail(fail(BMG_EDEVICE, "uploading the batch tables failed"));
    // every workgroup of the persistent launch must be resident at once
    if (hipFuncSetAttribute((const void *)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)B->lds) != hipSuccess)
        return bail(fail(BMG_EDEVICE, "cannot reserve %zu bytes of LDS", B->lds));
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch, BT, B->lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1)
        return bail(fail(BMG_EDEVICE, "occupancy query failed"));
    B->nblocks = per_cu * ncu;
    *out = B;
    return BMG_OK;
}

}  // extern "C"

namespace {

BArgs batch_args(const bmg_batch *B, double tol)
{
    BArgs A;
    A.P = B->dP;
    A.items = B->ditems;
    A.li = B->li;
    A.nprob = B->nprob;
    A.tol = tol;
    A.maxc = B->maxc;
    A.active = B->dactive;
    return A;
}

bmg_status batch_launch(bmg_batch *B, int mode, int steps, double tol)
{
    BArgs A = batch_args(B, tol);
    void *args[] = {&A, &mode, &steps};
    HIPCHK(hipLaunchCooperativeKernel((const void *)k_batch, dim3(B->nblocks), dim3(BT), args, B->lds, B->st));
    return BMG_OK;
}

// The launch of `steps` refinement steps as a HIP graph of one cooperative
// kernel node, built once per (steps, tol) and replayed; direct cooperative
// launches if the runtime cannot build it or runs the node without the grid
// barrier (the kernel then reports active = -1 before doing any work).
bmg_status batch_steps(bmg_batch *B, int steps, double tol)
{
    if (!B->graph_tried || B->graph_steps != steps || B->graph_tol != tol) {
        if (B->exec) { (void)hipGraphExecDestroy(B->exec); B->exec = nullptr; }
        if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
        B->graph_tried = true;
        B->graph_ok = false;
        B->graph_steps = steps;
        B->graph_tol = tol;
        hipGraph_t g = nullptr;
        if (!B->graph_refused && hipGraphCreate(&g, 0) == hipSuccess) {
            BArgs A = batch_args(B, tol);
            int mode = MODE_STEPS, st = steps;
            void *args[] = {&A, &mode, &st};
            hipKernelNodeParams p;
            memset(&p, 0, sizeof p);
            p.func = (void *)k_batch;
            p.gridDim = dim3(B->nblocks);
            p.blockDim = dim3(BT);
            p.sharedMemBytes = B->lds;
            p.kernelParams = args;
            hipKernelNodeAttrValue v;
            memset(&v, 0, sizeof v);
            v.cooperative = 1;
            hipGraphNode_t node = nullptr;
            if (hipGraphAddKernelNode(&node, g, nullptr, 0, &p) == hipSuccess &&
                hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v) == hipSuccess &&
                hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) == hipSuccess) {
                B->graph = g;
                B->graph_ok = true;
            } else {
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipGetLastError();
    }
    if (B->graph_ok) {
        HIPCHK(hipGraphLaunch(B->exec, B->st));
        return BMG_OK;
    }
    return batch_launch(B, MODE_STEPS, steps, tol);
}

}  // namespace

extern "C" {

bmg_status bmg_batch_solve(bmg_batch *B, const double *const *rhs, double *const *x, double tol,
                           int *steps_out, double *rel_res)
{
    if (!B || !rhs || !x) return fail(BMG_EINVAL, "NULL argument");
    if (!(tol >= 0.0)) return fail(BMG_EINVAL, "tol must be >= 0");
    // caller pointers into the problem table
    for (int p = 0; p < B->nprob; ++p) {
        if (!rhs[p] || !x[p]) return fail(BMG_EINVAL, "problem %d: NULL array", p);
        HIPCHK(hipMemcpyAsync((char *)(B->dP + p) + offsetof(BProb, rhs), &rhs[p], sizeof(double *),
                              hipMemcpyHostToDevice, B->st));
        HIPCHK(hipMemcpyAsync((char *)(B->dP + p) + offsetof(BProb, x), &x[p], sizeof(double *),
                              hipMemcpyHostToDevice, B->st));
    }
    TRY(batch_launch(B, MODE_INIT, 0, tol));
    const int per_launch = 8;
    int active = 1;
    for (int done_steps = 0; active > 0 && done_steps <= B->maxc; done_steps += per_launch) {
        const bool via_graph = B->graph_ok || !B->graph_tried;
        TRY(batch_steps(B, per_launch, tol));
        HIPCHK(hipMemcpyAsync(&active, B->dactive, sizeof(int), hipMemcpyDeviceToHost, B->st));
        HIPCHK(hipStreamSynchronize(B->st));
        if (active < 0) {
            if (!via_graph || !B->graph_ok) return fail(BMG_EDEVICE, "the persistent launch was not cooperative");
            // the graph node ran without a grid barrier and did nothing: use
            // direct launches from here on, and release the graph now
            B->graph_ok = false;
            B->graph_refused = true;
            if (B->exec) { (void)hipGraphExecDestroy(B->exec); B->exec = nullptr; }
            if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
            TRY(batch_launch(B, MODE_STEPS, per_launch, tol));
            HIPCHK(hipMemcpyAsync(&active, B->dactive, sizeof(int), hipMemcpyDeviceToHost, B->st));
            HIPCHK(hipStreamSynchronize(B->st));
            if (active < 0) return fail(BMG_EDEVICE, "the persistent launch was not cooperative");
        }
    }
    TRY(batch_launch(B, MODE_FINISH, 0, tol));
    std::vector<BProb> hp(B->nprob);
    HIPCHK(hipMemcpyAsync(hp.data(), B->dP, hp.size() * sizeof(BProb), hipMemcpyDeviceToHost, B->st));
    HIPCHK(hipStreamSynchronize(B->st));
    bmg_status st = BMG_OK;
    for (int p = 0; p < B->nprob; ++p) {
        const int steps = hp[p].done == 5 ? 0 : hp[p].count - 1;
        if (steps_out) steps_out[p] = steps;
        if (rel_res) {
            double v = 0.0;
            if (hp[p].count > 0)
                HIPCHK(hipMemcpy(&v, hp[p].hist + hp[p].count - 1, sizeof v, hipMemcpyDeviceToHost));
            rel_res[p] = v;
        }
        if (hp[p].done == 2 && st == BMG_OK) st = fail(BMG_EDIVERGED, "problem %d diverged", p);
        if (hp[p].done == 3 && st == BMG_OK) st = fail(BMG_ENOCONV, "problem %d did not converge", p);
    }
    return st;
}

bmg_status bmg_batch_history(bmg_batch *B, int p, double *hist, int cap, int *count)
{
    if (!B || p < 0 || p >= B->nprob || !count) return fail(BMG_EINVAL, "bad arguments");
    BProb q;
    HIPCHK(hipMemcpy(&q, B->dP + p, sizeof q, hipMemcpyDeviceToHost));
    *count = q.done == 5 ? 0 : q.count;
    if (hist && cap > 0 && *count > 0)
        HIPCHK(hipMemcpy(hist, q.hist, std::min(cap, *count) * sizeof(double), hipMemcpyDeviceToHost));
    return BMG_OK;
}

bmg_status bmg_batch_info(const bmg_batch *B, int *nblocks, int *graph_used)
{
    if (!B) return fail(BMG_EINVAL, "NULL handle");
    if (nblocks) *nblocks = B->nblocks;
    if (graph_used) *graph_used = B->graph_ok ? 1 : (B->graph_refused ? 2 : 0);
    return BMG_OK;
}

bmg_status bmg_batch_destroy(bmg_batch *B)
{
    if (!B) return BMG_OK;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (bmg_solver *h : B->sub) bmg_destroy(h);
    delete B;
    return BMG_OK;
}

}  // extern "C"
