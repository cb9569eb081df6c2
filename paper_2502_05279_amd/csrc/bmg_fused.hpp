// Fused, row-streaming passes of the V-cycle (gfx950).
//
// One workgroup of 256 lanes owns a strip of 256 grid columns (one column per
// lane, `hx` halo columns on each side computed redundantly) and a block of
// `ht` rows, and streams upward through it two rows (an even and an odd row) at
// a time.  Four-colour Gauss-Seidel is a row pipeline: colours 0 and 1 live on
// even rows and need only OLD odd rows, colours 2 and 3 live on odd rows and
// need the NEW even rows on both sides, so at each step sweep s updates even
// row e-2s and then odd row e-2s-1, and sweep s+1 trails sweep s by one step.
// The residual and the restriction trail the last sweep.  A tile starts its
// pipeline a few rows below its block (warm-up rows whose values are not
// written) and reads the iterate from an input buffer that no workgroup
// writes, so overlapping tiles never race; the result goes to a second buffer.
//
// u and the entries read at a neighbouring column (W, and SW, NW on nine-point
// levels) sit in LDS ring buffers of rows; O, S and b, read only in the
// thread's own column, sit in per-thread register windows that shift by two
// rows per step.  Every point is computed with exactly the expression and term
// order of the single-step kernels, so results are bitwise identical to them.
#pragma once

#include "bmg_kernels.hpp"

namespace bmg {

constexpr int FW = 256;  // lanes (= columns) per workgroup

// Ring-buffer slot of a row (rows may be slightly negative near the bottom).
template <int R>
__device__ __forceinline__ int slot(int row)
{
    if constexpr ((R & (R - 1)) == 0)
        return (row + 64 * R) & (R - 1);
    else
        return (row + 64 * R) % R;
}

// Tile of the XCD-aware launch: consecutive workgroup ids are dealt round-robin
// to the 8 XCDs, so ids are regrouped to give each XCD a contiguous run of
// neighbouring tiles (their halos then meet in the same L2).
__device__ __forceinline__ int tile_id(int ntiles)
{
    const int g = gridDim.x;          // multiple of 8
    const int per = g >> 3;
    const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    return t < ntiles ? t : -1;
}

struct TileGeo {
    int hx;       // halo columns on each side
    int ht;       // owned rows per tile
    int tiles_x;  // strips
    int ntiles;
    // several right-hand sides on one hierarchy: right-hand side k's u, b (and
    // the output) start k*ksf elements after the first's, its coarse-level u, b
    // k*ksc after, its stop flag k*kstop ints after and its norm partials
    // k*kpart doubles after
    int nrhs = 1, kstop = 0, kpart = 0;
    size_t ksf = 0, ksc = 0;
};

// Work item of this workgroup: tile `tid` of right-hand side `k`.  The nrhs
// workgroups of a tile get consecutive ids, so they run on the same XCD at
// about the same time and the stencil and weight rows they share are fetched
// into its L2 once.
__device__ __forceinline__ bool tile_work(const TileGeo &G, int &tid, int &k)
{
    const int w = tile_id(G.ntiles * G.nrhs);
    if (w < 0) return false;
    tid = w / G.nrhs;
    k = w - tid * G.nrhs;
    return true;
}

// Gauss-Seidel update of point (lane, row) from the LDS rings: the same terms in
// the same order as gs_point.
template <typename T, bool NINE, int RU>
__device__ __forceinline__ T gs_lds(const T *su, const T *sW, const T *sSW, const T *sNW, int lane,
                                    int row, T b, T O, T S, T Sn)
{
    const int r0 = slot<RU>(row) * FW + lane;
    const int rd = slot<RU>(row - 1) * FW + lane;
    const int ru = slot<RU>(row + 1) * FW + lane;
    T s = b;
    if (NINE) s -= sSW[r0] * su[rd - 1];
    s -= S * su[rd];
    if (NINE) s -= sNW[rd + 1] * su[rd + 1];
    s -= sW[r0] * su[r0 - 1];
    s -= sW[r0 + 1] * su[r0 + 1];
    if (NINE) s -= sNW[r0] * su[ru - 1];
    s -= Sn * su[ru];
    if (NINE) s -= sSW[ru + 1] * su[ru + 1];
    return s / O;
}

template <typename T, bool NINE, int RU>
__device__ __forceinline__ T res_lds(const T *su, const T *sW, const T *sSW, const T *sNW, int lane,
                                     int row, T b, T O, T S, T Sn)
{
    const int r0 = slot<RU>(row) * FW + lane;
    const int rd = slot<RU>(row - 1) * FW + lane;
    const int ru = slot<RU>(row + 1) * FW + lane;
    T s = b;
    if (NINE) s -= sSW[r0] * su[rd - 1];
    s -= S * su[rd];
    if (NINE) s -= sNW[rd + 1] * su[rd + 1];
    s -= sW[r0] * su[r0 - 1];
    s -= sW[r0 + 1] * su[r0 + 1];
    if (NINE) s -= sNW[r0] * su[ru - 1];
    s -= Sn * su[ru];
    if (NINE) s -= sSW[ru + 1] * su[ru + 1];
    s -= O * su[r0];
    return s;
}

// ----------------------------------------------------------- pre pass
// u_out = GS^NU(u_in); b_c = P^T (b - A u_out) on the coarse rows owned by the
// tile; u_c = 0 there.  Window: rows e-2NU-2 .. e+1 (RW rows) at step e.  All
// global data of step e+2 (rows e+2, e+3 and the weights of its restriction
// row) is requested before step e computes, so the loads overlap the compute.
// LDS of one pre/post tile (ring rows RU, nine-point rings only if NINE)
template <typename T, bool NINE, int NU, bool WREC = false>
struct TileLds {
    static constexpr int RW = 2 * NU + 4;
    static constexpr int RU = RW <= 8 ? 8 : 16;
    T su[RU * FW], sW[RU * FW], sx[4 * FW];
    // unused parts have length zero: four five-point FP64 tiles of 40 KiB
    // then share one CU's 160 KiB
    T sSW[NINE ? RU * FW : 0], sNW[NINE ? RU * FW : 0];
    // weights computed in the pass (WREC): y-edge LB, LA of the even columns
    // and six values of the odd columns, each indexed by lane / 2
    T wy[WREC ? FW : 0], wx[WREC ? 3 * FW : 0];
};

// A refinement step folded into the fine level's passes (five-point level,
// one right-hand side).  FP32 inner cycle: the pre pass starts from u = 0 and
// reads the FP64 residual r in place of b: b = fl32(r / s) with s = 2^e the
// least power of two >= ||r||_inf (the scaling of k_ir_scale), which it also
// stores as the FP32 right-hand side for the post pass and, from one lane,
// into scale[0].  The post pass (FP32 or FP64 inner cycle) adds s * u to the
// double-FP64 iterate (XH, XL) as each owned point's final value is produced,
// with the arithmetic of dd_update_point, in place of storing u; s = 1 when
// scale is null (FP64 inner cycle, where 1 * u = u exactly).
struct IrArgs {
    const double *r;     // FP64 residual, the level's pitch
    const double *rmax;  // ||r||_inf
    double *scale;       // s, written by the pre pass; null: s = 1
    double *XH, *XL;     // double-FP64 iterate
};

// The NU sweeps of a step on a five-point level, colours merged across rows.
// Colour c updates the columns with parity c & 1, colours 0, 1 on the step's
// even row e - 2s, colours 2, 3 on its odd row e - 2s - 1.  With five-point
// couplings colour 1 (odd i, even j) and colour 2 (even i, odd j) do not
// touch, nor do colour 3 of sweep s and colour 0 of sweep s + 1 (which trails
// two rows lower): each pair runs as one phase, every column busy, and every
// point still sees the neighbour values of the order 0, 1, 2, 3, so the
// result is the same to the bit.  Phases: c0(s=0); then per sweep
// {c1, c2(s)} and {c3(s), c0(s+1)}: 2 NU + 1 barriers instead of 4 NU.
// The window rows are compile-time positions k = row - (e - 2NU - 2); a lane
// picks its row's entries by its column parity.
// done(s) runs after the phase that completes sweep s (all lanes past the
// barrier that follows it).
template <typename T, int NU, int RU, typename Done>
__device__ __forceinline__ void five_point_sweeps(T *su, const T *sW, int lane, int i, bool col_upd, int n, int e,
                                                  const T *rB, const T *rO, const T *rS, Done &&done)
{
    const bool odd = i & 1;
    const int base = e - 2 * NU - 2;
    // the update of the point of this lane's column in window row k (if any)
    auto upd = [&](bool on, int k) {
        const int row = base + k;
        if (on && col_upd && row >= 1 && row <= n) {
            const T v = gs_lds<T, false, RU>(su, sW, nullptr, nullptr, lane, row, rB[k], rO[k], rS[k], rS[k + 1]);
            su[slot<RU>(row) * FW + lane] = v;
        }
    };
    // a phase where odd columns update window row ko and even columns row ke.
    // The entries of both rows are taken as values first (the empty asm keeps
    // them values): a select between two elements of a register array is
    // otherwise turned into one element at a per-lane index, a chain of a
    // select per array element for each half of each value, which was a fifth
    // of the fine pass's vector instructions.
    auto pick = [](T vo, T ve, bool odd_lane) {
        asm volatile("" : "+v"(vo), "+v"(ve));
        return odd_lane ? vo : ve;
    };
    auto pair = [&](bool on_odd, int ko, bool on_even, int ke) {
        const bool on = odd ? on_odd : on_even;
        const int row = base + (odd ? ko : ke);
        if (on && col_upd && row >= 1 && row <= n) {
            const T b = pick(rB[ko], rB[ke], odd);
            const T o = pick(rO[ko], rO[ke], odd);
            const T s0 = pick(rS[ko], rS[ke], odd);
            const T s1 = pick(rS[ko + 1], rS[ke + 1], odd);
            const T v = gs_lds<T, false, RU>(su, sW, nullptr, nullptr, lane, row, b, o, s0, s1);
            su[slot<RU>(row) * FW + lane] = v;
        }
    };
    upd(!odd, 2 * NU + 2);                                  // c0 of sweep 0 on row e
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NU; ++s) {
        const int ke = 2 * NU + 2 - 2 * s;                  // even row e - 2s
        pair(true, ke, true, ke - 1);                       // c1 on e - 2s, c2 on e - 2s - 1
        __syncthreads();
        pair(true, ke - 1, s + 1 < NU, ke - 2);             // c3 on e - 2s - 1, c0 of s + 1 on e - 2s - 2
        __syncthreads();
        done(s);
    }
}

template <typename T, int NU, int RU>
__device__ __forceinline__ void five_point_sweeps(T *su, const T *sW, int lane, int i, bool col_upd, int n, int e,
                                                  const T *rB, const T *rO, const T *rS)
{
    five_point_sweeps<T, NU, RU>(su, sW, lane, i, col_upd, n, e, rB, rO, rS, [](int) {});
}

// With WREC the restriction weights are not read: each column computes the
// operator-induced weights of its own F-points from the stencil rows in the
// window (the expressions of k_weights_edges / k_weights_corners in their
// order, so the same bits), and the restricting columns collect their
// neighbours' through LDS.  Step e computes the y-edges and cell centres of
// row e-2NU-1 and the x-edges of row e-2NU; the weights of the rows below come
// from the previous step.
template <typename T, bool NINE, int NU, bool WREC = false, bool IRIN = false>
__device__ __forceinline__ void pre_tile(const Lev<T> &L, T *__restrict__ uout, const Wts<T> &C,
                                         const Lev<T> &Cl, const TileGeo &G, int tid,
                                         TileLds<T, NINE, NU, WREC> &S, IrArgs ir = {})
{
    constexpr int RW = 2 * NU + 4;                 // window rows
    constexpr int RU = RW <= 8 ? 8 : 16;           // LDS ring rows (power of two)
    T *su = S.su, *sW = S.sW, *sr = S.sx, *sSW = S.sSW, *sNW = S.sNW;

    const int n = L.n, ld = L.ld, lane = threadIdx.x, nc = Cl.n;
    const int useful = FW - 2 * G.hx;
    const int tx = tid % G.tiles_x, ty = tid / G.tiles_x;
    const int x0 = 1 + tx * useful;                // first owned column
    const int i = x0 - G.hx + lane;                // this lane's column
    const bool col_in = i >= 0 && i <= n + 1;
    const bool col_upd = i >= 1 && i <= n && lane >= 1 && lane < FW - 1;
    const bool col_own = i >= x0 && i < x0 + useful && i <= n;
    const int y0 = 1 + ty * G.ht;                  // owned rows [y0, y1)
    const int y1 = min(y0 + G.ht, n + 1);
    const int es = (y0 - 2 * NU) & ~1;             // warm-up rows below y0 that make
                                                   // the owned rows and coarse rows exact
    const int jlast = (y1 - 1) >> 1;               // last owned coarse row
    const int elast = 2 * jlast + 2 * NU + 2;      // step that restricts it
    const int I = i >> 1;
    const bool restrictor = !(i & 1) && col_own && I >= 1 && I <= nc;

    T rO[RW], rS[RW], rB[RW];
    auto ld_row = [&](const T *a, int row) -> T {
        return (col_in && row >= 0 && row <= n + 1) ? a[(size_t)row * ld + i] : (T)0;
    };
    // the iterate and the right-hand side as the pass reads them (IRIN: zero,
    // and the scaled FP64 residual at interior points)
    double inv = 1.0;
    if constexpr (IRIN) {
        const int ex = ir_exponent(*ir.rmax);
        inv = ldexp(1.0, -ex);
        if (tid == 0 && lane == 0) ir.scale[0] = ldexp(1.0, ex);
    }
    auto ld_u = [&](int row) -> T { return IRIN ? (T)0 : ld_row(L.u, row); };
    auto ld_b = [&](int row) -> T {
        if constexpr (IRIN)
            return (i >= 1 && i <= n && row >= 1 && row <= n) ? (T)(ir.r[(size_t)row * ld + i] * inv) : (T)0;
        else
            return ld_row(L.b, row);
    };
    // the eight weights of coarse point (I, J) in the order the restriction uses
    auto ld_w = [&](int J, T w[8]) {
        const bool ok = restrictor && J >= 1 && J <= nc;
        const size_t c = ok ? (size_t)J * C.ld + I : 0, cn = c + C.ld;
        w[0] = ok ? C.at(LNE, c) : (T)0;
        w[1] = ok ? C.at(LA, c) : (T)0;
        w[2] = ok ? C.at(LNW, c + 1) : (T)0;
        w[3] = ok ? C.at(LR, c) : (T)0;
        w[4] = ok ? C.at(LL, c + 1) : (T)0;
        w[5] = ok ? C.at(LSE, cn) : (T)0;
        w[6] = ok ? C.at(LB, cn) : (T)0;
        w[7] = ok ? C.at(LSW, cn + 1) : (T)0;
    };
    // window of step es without its own two rows: rows es-2NU-2 .. es-1, placed
    // at positions 2..RW-1 so that the first shift by two aligns them
#pragma unroll
    for (int k = 2; k < RW; ++k) {
        const int row = es - 2 * NU - 4 + k;
        su[slot<RU>(row) * FW + lane] = ld_u(row);
        sW[slot<RU>(row) * FW + lane] = ld_row(L.W, row);
        if (NINE) {
            sSW[slot<RU>(row) * FW + lane] = ld_row(L.SW, row);
            sNW[slot<RU>(row) * FW + lane] = ld_row(L.NW, row);
        }
        rO[k] = ld_row(L.O, row);
        rS[k] = ld_row(L.S, row);
        rB[k] = ld_b(row);
    }
    // the lumped nine-point row of this column at window row k (WREC)
    auto row9 = [&](int k, int row, T a[9]) {
        const int r0 = slot<RU>(row) * FW + lane;
        a[0] = NINE ? sSW[r0] : (T)0;
        a[1] = rS[k];
        a[2] = NINE ? sNW[slot<RU>(row - 1) * FW + lane + 1] : (T)0;
        a[3] = sW[r0];
        a[4] = rO[k];
        a[5] = sW[r0 + 1];
        a[6] = NINE ? sNW[r0] : (T)0;
        a[7] = rS[k + 1];
        a[8] = NINE ? sSW[slot<RU>(row + 1) * FW + lane + 1] : (T)0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            if (q == 4) continue;
            if (a[q] > (T)0) {
                a[4] = a[4] + a[q];
                a[q] = (T)0;
            }
        }
    };
    // exchange index of this column: lanes and columns have opposite parity
    // (x0 - hx is odd: x0 = 1 + tx * useful with useful even, hx even), so the
    // odd columns' indices lane/2 are distinct, and so are the even columns'
    const int wl = lane >> 1;
    const bool odd_col = i & 1;
    // weights of the previous step (rows below) kept by their columns: odd
    // columns LNE, LNW of the centre and LR, LL of the x-edge, even columns LA
    T pLNE = 0, pLNW = 0, pLR = 0, pLL = 0, pLA = 0, yLB = 0, yLA = 0;

    // data of the first step
    T pu0, pu1, pW0, pW1, pO0, pO1, pS0, pS1, pB0, pB1, pSW0 = 0, pSW1 = 0, pNW0 = 0, pNW1 = 0;
    T pw[8], w[8];
    auto fetch = [&](int e) {
        pu0 = ld_u(e); pu1 = ld_u(e + 1);
        pW0 = ld_row(L.W, e); pW1 = ld_row(L.W, e + 1);
        pO0 = ld_row(L.O, e); pO1 = ld_row(L.O, e + 1);
        pS0 = ld_row(L.S, e); pS1 = ld_row(L.S, e + 1);
        pB0 = ld_b(e); pB1 = ld_b(e + 1);
        if (NINE) {
            pSW0 = ld_row(L.SW, e); pSW1 = ld_row(L.SW, e + 1);
            pNW0 = ld_row(L.NW, e); pNW1 = ld_row(L.NW, e + 1);
        }
        if (!WREC) ld_w((e - 2 * NU - 2) >> 1, pw);
        if (IRIN && col_own) {
            // every owned row is fetched once: keep its FP32 right-hand side
            if (e >= y0 && e < y1) L.b[(size_t)e * ld + i] = pB0;
            if (e + 1 >= y0 && e + 1 < y1) L.b[(size_t)(e + 1) * ld + i] = pB1;
        }
    };
    fetch(es);
    // restriction of the coarse row of step e (J = (e - 2NU - 2) / 2) by the
    // even columns, from the residual ring and the weights of step e (in w, or
    // with WREC in LDS); it runs after the next step's first barrier (or after
    // the last step), before anything overwrites them
    auto restrict_step = [&](int e) {
        if (WREC && restrictor) {
            // odd neighbours: i-1 at exchange index wl, i+1 at wl+1
            w[0] = S.wx[wl];                  // LNE of the centre (i-1, f-1)
            w[1] = pLA;                       // LA of the y-edge (i, f-1)
            w[2] = S.wx[FW / 2 + wl + 1];     // LNW of the centre (i+1, f-1)
            w[3] = S.wx[FW + wl];             // LR of the x-edge (i-1, f)
            w[4] = S.wx[3 * FW / 2 + wl + 1]; // LL of the x-edge (i+1, f)
            w[5] = S.wx[2 * FW + wl];         // LSE of the centre (i-1, f+1)
            w[6] = yLB;                       // LB of the y-edge (i, f+1)
            w[7] = S.wx[5 * FW / 2 + wl + 1]; // LSW of the centre (i+1, f+1)
        }
        if (WREC && !odd_col) pLA = yLA;
        const int f = e - 2 * NU - 2, J = f >> 1;
        if (restrictor && J >= 1 && J <= nc && f >= y0 && f < y1) {
            const size_t c = (size_t)J * C.ld + I;
            const T *rd = sr + ((f - 1) & 3) * FW + lane, *r0 = sr + (f & 3) * FW + lane,
                    *ru = sr + ((f + 1) & 3) * FW + lane;
            T s = w[0] * rd[-1];
            s = s + w[1] * rd[0];
            s = s + w[2] * rd[1];
            s = s + w[3] * r0[-1];
            s = s + r0[0];
            s = s + w[4] * r0[1];
            s = s + w[5] * ru[-1];
            s = s + w[6] * ru[0];
            s = s + w[7] * ru[1];
            Cl.b[c] = s;
            Cl.u[c] = (T)0;
        }
    };

    for (int e = es; e <= elast; e += 2) {
        __syncthreads();  // the previous step is done with the slots reused below
        if (e > es) restrict_step(e - 2);
        {
            const int s0 = slot<RU>(e) * FW + lane, s1 = slot<RU>(e + 1) * FW + lane;
            su[s0] = pu0; su[s1] = pu1;
            sW[s0] = pW0; sW[s1] = pW1;
            if (NINE) { sSW[s0] = pSW0; sSW[s1] = pSW1; sNW[s0] = pNW0; sNW[s1] = pNW1; }
#pragma unroll
            for (int k = 0; k < RW - 2; ++k) { rO[k] = rO[k + 2]; rS[k] = rS[k + 2]; rB[k] = rB[k + 2]; }
            rO[RW - 2] = pO0; rO[RW - 1] = pO1;
            rS[RW - 2] = pS0; rS[RW - 1] = pS1;
            rB[RW - 2] = pB0; rB[RW - 1] = pB1;
            if (!WREC) {
#pragma unroll
                for (int q = 0; q < 8; ++q) w[q] = pw[q];
            }
        }
        if (e + 2 <= elast) fetch(e + 2);
        __syncthreads();
        if (WREC && !odd_col) {
            // y-edge of row f+1 (f = e-2NU-2, window row 1): collapse along x;
            // zero where the F-point does not exist (the ring), as in the
            // stored planes
            const int row = e - 2 * NU - 1;
            yLB = yLA = (T)0;
            if (col_upd && row >= 1 && row <= n) {
                T a[9];
                row9(1, row, a);
                const T D = (a[4] + a[3]) + a[5];
                yLB = -((a[1] + a[0]) + a[2]) / D;
                yLA = -((a[7] + a[6]) + a[8]) / D;
            }
            S.wy[wl] = yLB;
            S.wy[FW / 2 + wl] = yLA;
        }
        // (the colour barriers below publish wy)
        // NU sweeps, each over colours 0,1 (even row) then 2,3 (odd row)
        if constexpr (NINE) {
#pragma unroll
            for (int s = 0; s < NU; ++s) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int row = c < 2 ? e - 2 * s : e - 2 * s - 1;
                    const int k = row - (e - 2 * NU - 2);
                    if (col_upd && (i & 1) == (c & 1) && row >= 1 && row <= n) {
                        const T v = gs_lds<T, NINE, RU>(su, sW, sSW, sNW, lane, row, rB[k], rO[k], rS[k], rS[k + 1]);
                        su[slot<RU>(row) * FW + lane] = v;
                    }
                    __syncthreads();
                }
            }
        } else {
            five_point_sweeps<T, NU, RU>(su, sW, lane, i, col_upd, n, e, rB, rO, rS);
        }
        // the last sweep's two rows are final: write the owned ones
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int row = e - 2 * NU + 2 - t;
            if (col_own && row >= y0 && row < y1)
                uout[(size_t)row * ld + i] = su[slot<RU>(row) * FW + lane];
        }
        if (WREC && col_upd && odd_col) {
            // x-edge of row f+2 (window row 2): collapse along y (zero on the ring)
            T a[9];
            T xLL = (T)0, xLR = (T)0;
            if (e - 2 * NU >= 1 && e - 2 * NU <= n) {
                row9(2, e - 2 * NU, a);
                const T D = (a[4] + a[7]) + a[1];
                xLL = -((a[3] + a[6]) + a[0]) / D;
                xLR = -((a[5] + a[8]) + a[2]) / D;
            }
            // cell centre of row f+1 from its own row and the edges around it
            row9(1, e - 2 * NU - 1, a);
            const T lbw = S.wy[wl - 1], law = S.wy[FW / 2 + wl - 1];
            const T lbe = S.wy[wl], lae = S.wy[FW / 2 + wl];
            const T cLNE = -((a[8] + a[7] * xLR) + a[5] * lae) / a[4];
            const T cLNW = -((a[6] + a[7] * xLL) + a[3] * law) / a[4];
            const T cLSE = -((a[2] + a[1] * pLR) + a[5] * lbe) / a[4];
            const T cLSW = -((a[0] + a[1] * pLL) + a[3] * lbw) / a[4];
            S.wx[wl] = pLNE;
            S.wx[FW / 2 + wl] = pLNW;
            S.wx[FW + wl] = pLR;
            S.wx[3 * FW / 2 + wl] = pLL;
            S.wx[2 * FW + wl] = cLSE;
            S.wx[5 * FW / 2 + wl] = cLSW;
            pLNE = cLNE; pLNW = cLNW; pLR = xLR; pLL = xLL;
        }
        // residual of rows e-2NU and e-2NU-1
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int row = e - 2 * NU - t;
            const int k = row - (e - 2 * NU - 2);
            T r = 0;
            if (col_upd && row >= 1 && row <= n)
                r = res_lds<T, NINE, RU>(su, sW, sSW, sNW, lane, row, rB[k], rO[k], rS[k], rS[k + 1]);
            sr[(row & 3) * FW + lane] = r;
        }
    }
    __syncthreads();
    restrict_step(elast);
}

template <typename T, bool NINE, int NU, bool WREC = false>
__global__ __launch_bounds__(FW) void k_pre(Lev<T> L, T *__restrict__ uout, Wts<T> C, Lev<T> Cl,
                                             TileGeo G, const int *stop)
{
    int tid, k;
    if (!tile_work(G, tid, k)) return;
    if (stopped(stop ? stop + k * G.kstop : stop)) return;
    L.u += k * G.ksf; L.b += k * G.ksf; uout += k * G.ksf;
    Cl.u += k * G.ksc; Cl.b += k * G.ksc;
    __shared__ TileLds<T, NINE, NU, WREC> S;
    pre_tile<T, NINE, NU, WREC>(L, uout, C, Cl, G, tid, S);
}

// ---------------------------------------------------------- post pass
// u_out = GS^NU(u_in + P e_c).  With NORM (FP64 fine level) also the
// per-tile sum of squares of the accurate residual b - A u_out over the owned
// points into part[tile].  Window: rows e-2NU-2 .. e+1 at step e; the data of
// step e+2 (rows, coarse row, interpolation weights) is requested while step
// e computes.
template <typename T, bool NINE, int NU, bool NORM, bool IRUP = false>
__device__ __forceinline__ void post_tile(const Lev<T> &L, T *__restrict__ uout, const Wts<T> &C,
                                          const T *__restrict__ ec, const TileGeo &G, int tid,
                                          double *__restrict__ part, TileLds<T, NINE, NU> &S, IrArgs ir = {})
{
    static_assert(NU <= 2, "post pass supports up to two sweeps");
    constexpr int RW = 2 * NU + 4;
    constexpr int RU = RW <= 8 ? 8 : 16;
    T *su = S.su, *sW = S.sW, *sec = S.sx, *sSW = S.sSW, *sNW = S.sNW;

    const int n = L.n, ld = L.ld, lane = threadIdx.x, ldc = C.ld, nc = (n - 1) >> 1;
    const int useful = FW - 2 * G.hx;
    const int tx = tid % G.tiles_x, ty = tid / G.tiles_x;
    const int x0 = 1 + tx * useful;
    const int i = x0 - G.hx + lane;
    const bool col_in = i >= 0 && i <= n + 1;
    const bool col_upd = i >= 1 && i <= n && lane >= 1 && lane < FW - 1;
    const bool col_own = i >= x0 && i < x0 + useful && i <= n;
    const int y0 = 1 + ty * G.ht;
    const int y1 = min(y0 + G.ht, n + 1);
    const int es = (y0 - 2 * NU + 1) & ~1;         // warm-up rows below y0
    const int elast = ((y1 + 2 * NU) + 1) & ~1;    // the norm reaches row y1 - 1
    // coarse columns of this strip in LDS: I = ib + lane
    const int ib = (x0 - G.hx) >> 1;
    const int Ie = ib + lane;
    const bool ccol_in = lane < FW / 2 + 2 && Ie >= 0 && Ie <= nc + 1;
    const bool odd_i = i & 1;
    const int Ix = (i + 1) >> 1;                   // coarse column east of an odd column

    T rO[RW], rS[RW], rB[RW];
    auto ld_row = [&](const T *a, int row) -> T {
        return (col_in && row >= 0 && row <= n + 1) ? a[(size_t)row * ld + i] : (T)0;
    };
    auto ld_crow = [&](int J) -> T {
        return (ccol_in && J >= 0 && J <= nc + 1) ? ec[(size_t)J * ldc + Ie] : (T)0;
    };
    // interpolation weights of this column for fine rows e (even) and e+1 (odd):
    // odd columns: LL, LR at (Ix, e/2), then LSW, LSE, LNW, LNE at (Ix, e/2+1);
    // even columns: LB, LA at (i/2, e/2+1)
    struct IW { T w[6]; };
    // the planes this column reads for its odd row: LSW, LSE, LNW, LNE (odd
    // columns) or LB, LA (even columns); every lane issues the same six loads
    const int p2 = odd_i ? LSW : LB, p3 = odd_i ? LSE : LA;
    auto ld_iw = [&](int e) -> IW {
        IW r;
        T *w = r.w;
        const int J0 = e >> 1, J1 = J0 + 1;
        const bool ok0 = col_upd && odd_i && e >= 1 && e <= n;
        const bool ok1 = col_upd && e + 1 >= 1 && e + 1 <= n;
        const bool ok2 = ok1 && odd_i;
        const size_t c0 = ok0 ? (size_t)J0 * ldc + Ix : 0;
        const size_t c1 = ok1 ? (size_t)J1 * ldc + (odd_i ? Ix : (i >> 1)) : 0;
        w[0] = ok0 ? C.at(LL, c0) : (T)0;
        w[1] = ok0 ? C.at(LR, c0) : (T)0;
        w[2] = ok1 ? C.at(p2, c1) : (T)0;
        w[3] = ok1 ? C.at(p3, c1) : (T)0;
        w[4] = ok2 ? C.at(LNW, c1) : (T)0;
        w[5] = ok2 ? C.at(LNE, c1) : (T)0;
        return r;
    };
    // u + P e_c at (i, row) for an even (row = e) or odd (row = e+1) row, with
    // the weights w of ld_iw and e_c from the LDS ring
    auto interp = [&](int row, T u, const IW &iw) -> T {
        const T *w = iw.w;
        if (!col_upd || row < 1 || row > n) return u;
        T e;
        if (!(row & 1)) {
            const T *er = sec + ((row >> 1) & 3) * FW;
            if (!odd_i) e = er[(i >> 1) - ib];
            else e = w[0] * er[Ix - 1 - ib] + w[1] * er[Ix - ib];
        } else {
            const int J = (row + 1) >> 1;
            const T *es_ = sec + ((J - 1) & 3) * FW, *en = sec + (J & 3) * FW;
            if (!odd_i) {
                e = w[2] * es_[(i >> 1) - ib] + w[3] * en[(i >> 1) - ib];
            } else {
                e = w[2] * es_[Ix - 1 - ib] + w[3] * es_[Ix - ib];
                e = e + w[4] * en[Ix - 1 - ib];
                e = e + w[5] * en[Ix - ib];
            }
        }
        return u + e;
    };

    // window of step es without its own two rows: rows es-2NU-2 .. es-1,
    // interpolated, at positions 2..RW-1 (aligned by the first shift); their
    // coarse rows are (es-2NU-2)/2 .. es/2, at most four (the e_c ring)
    for (int J = (es - 2 * NU - 2) >> 1; J <= (es >> 1); ++J) sec[(J & 3) * FW + lane] = ld_crow(J);
    __syncthreads();
#pragma unroll
    for (int k = 2; k < RW; k += 2) {
        const int row = es - 2 * NU - 4 + k;      // even
        const IW wk = ld_iw(row);
        su[slot<RU>(row) * FW + lane] = interp(row, ld_row(L.u, row), wk);
        su[slot<RU>(row + 1) * FW + lane] = interp(row + 1, ld_row(L.u, row + 1), wk);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            sW[slot<RU>(row + t) * FW + lane] = ld_row(L.W, row + t);
            if (NINE) {
                sSW[slot<RU>(row + t) * FW + lane] = ld_row(L.SW, row + t);
                sNW[slot<RU>(row + t) * FW + lane] = ld_row(L.NW, row + t);
            }
            rO[k + t] = ld_row(L.O, row + t);
            rS[k + t] = ld_row(L.S, row + t);
            rB[k + t] = ld_row(L.b, row + t);
        }
    }
    // coarse row es/2 + 1, which the first step reads with es/2; from then on
    // each step writes the row two steps ahead of its own, so that no step
    // reads a row written in it
    {
        const T v = ld_crow((es >> 1) + 1);
        __syncthreads();
        sec[(((es >> 1) + 1) & 3) * FW + lane] = v;
        __syncthreads();
    }
    T pu0, pu1, pW0, pW1, pO0, pO1, pS0, pS1, pB0, pB1, pSW0 = 0, pSW1 = 0, pNW0 = 0, pNW1 = 0, pec;
    IW pw;
    // IRUP: the double-FP64 iterate at the two rows a step finalises (rows
    // e-2NU+2 and e-2NU+1 at step e), requested one step ahead
    const double sc = IRUP ? (ir.scale ? *ir.scale : 1.0) : 0.0;
    auto owned = [&](int row) { return col_own && row >= y0 && row < y1; };
    double xh[2] = {0.0, 0.0}, xl[2] = {0.0, 0.0}, pxh[2] = {0.0, 0.0}, pxl[2] = {0.0, 0.0};
    auto fetch = [&](int e) {
        if (IRUP) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int row = e - 2 * NU + 2 - t;
                const size_t p = (size_t)row * ld + i;
                pxh[t] = owned(row) ? ir.XH[p] : 0.0;
                pxl[t] = owned(row) ? ir.XL[p] : 0.0;
            }
        }
        pu0 = ld_row(L.u, e); pu1 = ld_row(L.u, e + 1);
        pW0 = ld_row(L.W, e); pW1 = ld_row(L.W, e + 1);
        pO0 = ld_row(L.O, e); pO1 = ld_row(L.O, e + 1);
        pS0 = ld_row(L.S, e); pS1 = ld_row(L.S, e + 1);
        pB0 = ld_row(L.b, e); pB1 = ld_row(L.b, e + 1);
        if (NINE) {
            pSW0 = ld_row(L.SW, e); pSW1 = ld_row(L.SW, e + 1);
            pNW0 = ld_row(L.NW, e); pNW1 = ld_row(L.NW, e + 1);
        }
        pec = ld_crow((e >> 1) + 2);
        pw = ld_iw(e);
    };
    fetch(es);
    double acc = 0.0;
    for (int e = es; e <= elast; e += 2) {
        // with two ring rows beyond the window the rows this step brings in
        // take slots no lane still reads, and no barrier is needed before them
        if constexpr (RU - RW < 2) __syncthreads();
        // coarse row e/2 + 2 joins the e_c ring for the next step (this step
        // reads rows e/2 and e/2 + 1; the slot is that of e/2 - 2)
        sec[(((e >> 1) + 2) & 3) * FW + lane] = pec;
#pragma unroll
        for (int k = 0; k < RW - 2; ++k) { rO[k] = rO[k + 2]; rS[k] = rS[k + 2]; rB[k] = rB[k + 2]; }
        rO[RW - 2] = pO0; rO[RW - 1] = pO1;
        rS[RW - 2] = pS0; rS[RW - 1] = pS1;
        rB[RW - 2] = pB0; rB[RW - 1] = pB1;
        if (IRUP) {
#pragma unroll
            for (int t = 0; t < 2; ++t) { xh[t] = pxh[t]; xl[t] = pxl[t]; }
        }
        {
            const int s0 = slot<RU>(e) * FW + lane, s1 = slot<RU>(e + 1) * FW + lane;
            su[s0] = interp(e, pu0, pw);
            su[s1] = interp(e + 1, pu1, pw);
            sW[s0] = pW0; sW[s1] = pW1;
            if (NINE) { sSW[s0] = pSW0; sSW[s1] = pSW1; sNW[s0] = pNW0; sNW[s1] = pNW1; }
        }
        if (e + 2 <= elast) fetch(e + 2);
        __syncthreads();
        if constexpr (NINE) {
#pragma unroll
            for (int s = 0; s < NU; ++s) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int row = c < 2 ? e - 2 * s : e - 2 * s - 1;
                    const int k = row - (e - 2 * NU - 2);
                    if (col_upd && (i & 1) == (c & 1) && row >= 1 && row <= n) {
                        const T v = gs_lds<T, NINE, RU>(su, sW, sSW, sNW, lane, row, rB[k], rO[k], rS[k], rS[k + 1]);
                        su[slot<RU>(row) * FW + lane] = v;
                    }
                    __syncthreads();
                }
            }
        } else {
            five_point_sweeps<T, NU, RU>(su, sW, lane, i, col_upd, n, e, rB, rO, rS);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int row = e - 2 * NU + 2 - t;
            if (owned(row)) {
                const size_t p = (size_t)row * ld + i;
                const T v = su[slot<RU>(row) * FW + lane];
                if constexpr (IRUP) {
                    // (XH, XL) += s v: TwoSum, add the low part, renormalise
                    const double d = sc * (double)v;
                    double hs, he;
                    two_sum(xh[t], d, hs, he);
                    he = he + xl[t];
                    const double hi = hs + he;
                    ir.XL[p] = he - (hi - hs);
                    ir.XH[p] = hi;
                } else {
                    uout[p] = v;
                }
            }
        }
        if (NORM) {
            // accurate residual of the final rows e-2NU and e-2NU-1
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int row = e - 2 * NU - t;
                const int k = row - (e - 2 * NU - 2);
                if (col_own && row >= y0 && row < y1 && row >= 1) {
                    const int r0 = slot<RU>(row) * FW + lane, rd = slot<RU>(row - 1) * FW + lane,
                              ru = slot<RU>(row + 1) * FW + lane;
                    double a[9], x[9];
                    a[0] = NINE ? (double)sSW[r0] : 0.0;        x[0] = su[rd - 1];
                    a[1] = rS[k];                               x[1] = su[rd];
                    a[2] = NINE ? (double)sNW[rd + 1] : 0.0;    x[2] = su[rd + 1];
                    a[3] = sW[r0];                              x[3] = su[r0 - 1];
                    a[4] = sW[r0 + 1];                          x[4] = su[r0 + 1];
                    a[5] = NINE ? (double)sNW[r0] : 0.0;        x[5] = su[ru - 1];
                    a[6] = rS[k + 1];                           x[6] = su[ru];
                    a[7] = NINE ? (double)sSW[ru + 1] : 0.0;    x[7] = su[ru + 1];
                    a[8] = rO[k];                               x[8] = su[r0];
                    double s = rB[k], cc = 0.0, ns, se;
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        if (!NINE && (q == 0 || q == 2 || q == 5 || q == 7)) continue;
                        const double pr = a[q] * x[q];
                        const double pe = fma(a[q], x[q], -pr);
                        two_sum(s, -pr, ns, se);
                        s = ns;
                        cc = cc + (se - pe);
                    }
                    const double r = s + cc;
                    acc += r * r;
                }
            }
        }
    }
    if (NORM) {
        __syncthreads();  // the residual ring is free again: reduce through it
        acc = block_sum(acc, reinterpret_cast<double *>(S.sx));
        if (threadIdx.x == 0) part[tid] = acc;
    }
}

template <typename T, bool NINE, int NU, bool NORM>
__global__ __launch_bounds__(FW) void k_post(Lev<T> L, T *__restrict__ uout, Wts<T> C, const T *__restrict__ ec,
                                              TileGeo G, double *__restrict__ part, const int *stop)
{
    int tid, k;
    if (!tile_work(G, tid, k)) return;
    if (stopped(stop ? stop + k * G.kstop : stop)) return;
    L.u += k * G.ksf; L.b += k * G.ksf; uout += k * G.ksf;
    ec += k * G.ksc;
    if (NORM) part += k * G.kpart;
    __shared__ TileLds<T, NINE, NU> S;
    post_tile<T, NINE, NU, NORM>(L, uout, C, ec, G, tid, part, S);
}

// --------------------------------- post pass and the next cycle's pre pass
// The fine level's post pass of cycle k and its pre pass of cycle k+1 as one
// pass (FP64, five-point level, one right-hand side, one post sweep, NB pre
// sweeps).  Rows enter as u' + P e_c; sweep 0 gives the cycle's result u_k,
// which is written (a stop decided by its norm finds it) and copied to a
// four-row LDS ring, from which the per-tile sum of squares of its accurate
// residual goes to part[tile]; sweeps 1..NB give the next cycle's
// pre-smoothed iterate u'' (written), whose residual is restricted with the
// stored weights (the rows the interpolation read, requested again).  Every array
// value is the one the two separate passes give (the norm's partial sums follow
// this pass's tiles).  u_c = 0 goes to a separate coarse buffer (ucz), since the
// coarse correction e_c is still read by other tiles.
template <int NB>
struct PostPreLds {
    static constexpr int NS = NB + 1;
    static constexpr int RW = 2 * NS + 4;
    static constexpr int RU = RW + 2;      // ring rows (see postpre_tile)
    static constexpr int CW = FW / 2 + 2;  // coarse columns of a strip
    double su[RU * FW], sW[RU * FW], sx[4 * FW];
    double sec[8 * CW];                    // e_c rows, ring of 8
    double uk[4 * FW];                     // u_k rows, ring of 4
};

template <int NB>
__device__ __forceinline__ void postpre_tile(const Lev<double> &L, double *__restrict__ ukout,
                                             double *__restrict__ uout, const Wts<double> &C,
                                             const double *__restrict__ ec, const Lev<double> &Cl,
                                             double *__restrict__ ucz, const TileGeo &G, int tid,
                                             double *__restrict__ part, PostPreLds<NB> &S)
{
    using T = double;
    constexpr int NS = NB + 1;                     // sweeps: one post, NB pre
    constexpr int RW = 2 * NS + 4;                 // window rows e-2NS-2 .. e+1
    // LDS ring rows: two more than the window, so that the rows a step
    // brings in take the slots of rows no step still reads, and a step needs
    // no barrier before writing them (the previous step's residuals read its
    // whole window)
    constexpr int RU = PostPreLds<NB>::RU;
    constexpr int CW = PostPreLds<NB>::CW;
    T *su = S.su, *sW = S.sW, *sr = S.sx, *sec = S.sec, *suk = S.uk;

    const int n = L.n, ld = L.ld, lane = threadIdx.x, nc = Cl.n, ldc = C.ld;
    const int useful = FW - 2 * G.hx;
    const int tx = tid % G.tiles_x, ty = tid / G.tiles_x;
    const int x0 = 1 + tx * useful;
    const int i = x0 - G.hx + lane;
    const bool col_in = i >= 0 && i <= n + 1;
    const bool col_upd = i >= 1 && i <= n && lane >= 1 && lane < FW - 1;
    const bool col_own = i >= x0 && i < x0 + useful && i <= n;
    const int y0 = 1 + ty * G.ht;
    const int y1 = min(y0 + G.ht, n + 1);
    const int es = (y0 - 2 * NS) & ~1;
    const int jlast = (y1 - 1) >> 1;
    const int elast = 2 * jlast + 2 * NS + 2;
    const int I = i >> 1;
    const bool restrictor = !(i & 1) && col_own && I >= 1 && I <= nc;
    const int ib = (x0 - G.hx) >> 1;               // coarse column of ring entry 0
    const int Ie = ib + lane;
    const bool ccol_in = lane < CW && Ie >= 0 && Ie <= nc + 1;
    const bool odd_i = i & 1;
    const int Ix = (i + 1) >> 1;

    T rO[RW], rS[RW], rB[RW];
    auto ld_row = [&](const T *a, int row) -> T {
        return (col_in && row >= 0 && row <= n + 1) ? a[(size_t)row * ld + i] : (T)0;
    };
    auto ld_crow = [&](int J) -> T {
        return (ccol_in && J >= 0 && J <= nc + 1) ? ec[(size_t)J * ldc + Ie] : (T)0;
    };
    // interpolation weights of this column for rows e (even) and e+1 (odd),
    // as in post_tile
    struct IW { T w[6]; };
    const int p2 = odd_i ? LSW : LB, p3 = odd_i ? LSE : LA;
    auto ld_iw = [&](int e) -> IW {
        IW r;
        T *w = r.w;
        const int J0 = e >> 1, J1 = J0 + 1;
        const bool ok0 = col_upd && odd_i && e >= 1 && e <= n;
        const bool ok1 = col_upd && e + 1 >= 1 && e + 1 <= n;
        const bool ok2 = ok1 && odd_i;
        const size_t c0 = ok0 ? (size_t)J0 * ldc + Ix : 0;
        const size_t c1 = ok1 ? (size_t)J1 * ldc + (odd_i ? Ix : (i >> 1)) : 0;
        w[0] = ok0 ? C.at(LL, c0) : (T)0;
        w[1] = ok0 ? C.at(LR, c0) : (T)0;
        w[2] = ok1 ? C.at(p2, c1) : (T)0;
        w[3] = ok1 ? C.at(p3, c1) : (T)0;
        w[4] = ok2 ? C.at(LNW, c1) : (T)0;
        w[5] = ok2 ? C.at(LNE, c1) : (T)0;
        return r;
    };
    // u' + P e_c at (i, row), e_c from the ring (the terms of post_tile)
    auto interp = [&](int row, T u, const IW &iw) -> T {
        const T *w = iw.w;
        if (!col_upd || row < 1 || row > n) return u;
        T e;
        if (!(row & 1)) {
            const T *er = sec + ((row >> 1) & 7) * CW;
            if (!odd_i) e = er[(i >> 1) - ib];
            else e = w[0] * er[Ix - 1 - ib] + w[1] * er[Ix - ib];
        } else {
            const int J = (row + 1) >> 1;
            const T *es_ = sec + ((J - 1) & 7) * CW, *en = sec + (J & 7) * CW;
            if (!odd_i) {
                e = w[2] * es_[(i >> 1) - ib] + w[3] * en[(i >> 1) - ib];
            } else {
                e = w[2] * es_[Ix - 1 - ib] + w[3] * es_[Ix - ib];
                e = e + w[4] * en[Ix - 1 - ib];
                e = e + w[5] * en[Ix - ib];
            }
        }
        return u + e;
    };

    // coarse rows of the first step's window and of the first two steps:
    // (es-2NS-2)/2 .. es/2 + 1 (NS + 3 <= 8 rows)
    for (int J = (es - 2 * NS - 2) >> 1; J <= (es >> 1) + 1; ++J) {
        const T v = ld_crow(J);
        if (lane < CW) sec[(J & 7) * CW + lane] = v;
    }
    __syncthreads();
    // window of step es without its own two rows: rows es-2NS-2 .. es-1,
    // interpolated, at positions 2..RW-1 (aligned by the first shift)
#pragma unroll
    for (int k = 2; k < RW; k += 2) {
        const int row = es - 2 * NS - 4 + k;       // even
        const IW wk = ld_iw(row);
        su[slot<RU>(row) * FW + lane] = interp(row, ld_row(L.u, row), wk);
        su[slot<RU>(row + 1) * FW + lane] = interp(row + 1, ld_row(L.u, row + 1), wk);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            sW[slot<RU>(row + t) * FW + lane] = ld_row(L.W, row + t);
            rO[k + t] = ld_row(L.O, row + t);
            rS[k + t] = ld_row(L.S, row + t);
            rB[k + t] = ld_row(L.b, row + t);
        }
    }
    // the stored weights of the coarse point a restriction step takes, as
    // k_restrict reads them (even columns that own a coarse point): requested
    // during step e, used when the restriction of step e runs after the first
    // barrier of step e + 2.  The post pass read the same rows four steps before, so
    // they come from the caches; computing them here instead (two lumped
    // rows and eight divisions per coarse point, in branches the odd and the
    // even columns each take) cost more time than the loads.
    T rw[8];
    auto fetch_rw = [&](int e) {
        const int J = (e - 2 * NS - 2) >> 1;
        const bool ok = restrictor && J >= 1 && J <= nc;
        const size_t c = ok ? (size_t)J * ldc + I : 0, cn = c + ldc;
        rw[0] = ok ? C.at(LNE, c) : (T)0;
        rw[1] = ok ? C.at(LA, c) : (T)0;
        rw[2] = ok ? C.at(LNW, c + 1) : (T)0;
        rw[3] = ok ? C.at(LR, c) : (T)0;
        rw[4] = ok ? C.at(LL, c + 1) : (T)0;
        rw[5] = ok ? C.at(LSE, cn) : (T)0;
        rw[6] = ok ? C.at(LB, cn) : (T)0;
        rw[7] = ok ? C.at(LSW, cn + 1) : (T)0;
    };

    T pu0, pu1, pW0, pW1, pO0, pO1, pS0, pS1, pB0, pB1, pec;
    IW pw;
    // data of step e; the e_c row it adds is the one step e + 2 needs
    auto fetch = [&](int e) {
        pu0 = ld_row(L.u, e); pu1 = ld_row(L.u, e + 1);
        pW0 = ld_row(L.W, e); pW1 = ld_row(L.W, e + 1);
        pO0 = ld_row(L.O, e); pO1 = ld_row(L.O, e + 1);
        pS0 = ld_row(L.S, e); pS1 = ld_row(L.S, e + 1);
        pB0 = ld_row(L.b, e); pB1 = ld_row(L.b, e + 1);
        pec = ld_crow((e >> 1) + 2);
        pw = ld_iw(e);
    };
    fetch(es);
    double acc = 0.0;
    // restriction of the coarse row of step e (J = (e - 2NS - 2) / 2) by the
    // even columns, from the residual ring and the weights step e requested;
    // it runs after the next step's first barrier (or after the last step),
    // before that step's residuals overwrite the ring
    auto restrict_step = [&](int e) {
        const T *w = rw;
        const int f = e - 2 * NS - 2, J = f >> 1;
        if (restrictor && J >= 1 && J <= nc && f >= y0 && f < y1) {
            const size_t c = (size_t)J * Cl.ld + I;
            const T *rd = sr + ((f - 1) & 3) * FW + lane, *r0 = sr + (f & 3) * FW + lane,
                    *ru = sr + ((f + 1) & 3) * FW + lane;
            T s = w[0] * rd[-1];
            s = s + w[1] * rd[0];
            s = s + w[2] * rd[1];
            s = s + w[3] * r0[-1];
            s = s + r0[0];
            s = s + w[4] * r0[1];
            s = s + w[5] * ru[-1];
            s = s + w[6] * ru[0];
            s = s + w[7] * ru[1];
            Cl.b[c] = s;
            ucz[c] = (T)0;
        }
    };

    for (int e = es; e <= elast; e += 2) {
        if (lane < CW) sec[(((e >> 1) + 2) & 7) * CW + lane] = pec;
#pragma unroll
        for (int k = 0; k < RW - 2; ++k) { rO[k] = rO[k + 2]; rS[k] = rS[k + 2]; rB[k] = rB[k + 2]; }
        rO[RW - 2] = pO0; rO[RW - 1] = pO1;
        rS[RW - 2] = pS0; rS[RW - 1] = pS1;
        rB[RW - 2] = pB0; rB[RW - 1] = pB1;
        {
            const int s0 = slot<RU>(e) * FW + lane, s1 = slot<RU>(e + 1) * FW + lane;
            su[s0] = interp(e, pu0, pw);
            su[s1] = interp(e + 1, pu1, pw);
            sW[s0] = pW0; sW[s1] = pW1;
        }
        if (e + 2 <= elast) fetch(e + 2);
        __syncthreads();
        if (e > es) restrict_step(e - 2);
        fetch_rw(e);
        // sweep 0 completes rows e and e-1 of u_k: written, and kept for the norm
        five_point_sweeps<T, NS, RU>(su, sW, lane, i, col_upd, n, e, rB, rO, rS, [&](int s) {
            if (s == 0) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int row = e - t;
                    const T v = su[slot<RU>(row) * FW + lane];
                    suk[(row & 3) * FW + lane] = v;
                    if (col_own && row >= y0 && row < y1) ukout[(size_t)row * ld + i] = v;
                }
            }
        });
        // the last sweep's two rows are final: write the owned ones
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int row = e - 2 * NS + 2 - t;
            if (col_own && row >= y0 && row < y1)
                uout[(size_t)row * ld + i] = su[slot<RU>(row) * FW + lane];
        }
        // residual of rows e-2NS and e-2NS-1
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int row = e - 2 * NS - t;
            const int k = row - (e - 2 * NS - 2);
            T r = 0;
            if (col_upd && row >= 1 && row <= n)
                r = res_lds<T, false, RU>(su, sW, nullptr, nullptr, lane, row, rB[k], rO[k], rS[k], rS[k + 1]);
            sr[(row & 3) * FW + lane] = r;
        }
        // accurate residual of u_k at rows e-1 and e-2 (the terms of post_tile)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int row = e - 1 - t;
            const int k = row - (e - 2 * NS - 2);
            if (col_own && row >= y0 && row < y1 && row >= 1) {
                const int r0 = slot<RU>(row) * FW + lane;
                const T *xd = suk + ((row - 1) & 3) * FW + lane, *x0_ = suk + (row & 3) * FW + lane,
                        *xu = suk + ((row + 1) & 3) * FW + lane;
                double a[5], x[5];
                a[0] = rS[k];       x[0] = xd[0];
                a[1] = sW[r0];      x[1] = x0_[-1];
                a[2] = sW[r0 + 1];  x[2] = x0_[1];
                a[3] = rS[k + 1];   x[3] = xu[0];
                a[4] = rO[k];       x[4] = x0_[0];
                double s = rB[k], cc = 0.0, ns, se;
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const double pr = a[q] * x[q];
                    const double pe = fma(a[q], x[q], -pr);
                    two_sum(s, -pr, ns, se);
                    s = ns;
                    cc = cc + (se - pe);
                }
                const double r = s + cc;
                acc += r * r;
            }
        }
    }
    __syncthreads();
    restrict_step(elast);
    __syncthreads();  // the residual ring is free again: reduce through it
    acc = block_sum(acc, reinterpret_cast<double *>(S.sx));
    if (threadIdx.x == 0) part[tid] = acc;
}

template <int NB>
__global__ __launch_bounds__(FW) void k_postpre(Lev<double> L, double *__restrict__ ukout, double *__restrict__ uout,
                                                 Wts<double> C, const double *__restrict__ ec, Lev<double> Cl,
                                                 double *__restrict__ ucz, TileGeo G, double *__restrict__ part,
                                                 const int *stop)
{
    int tid, k;
    if (!tile_work(G, tid, k)) return;
    if (stopped(stop)) return;
    __shared__ PostPreLds<NB> S;
    postpre_tile<NB>(L, ukout, uout, C, ec, Cl, ucz, G, tid, part, S);
}

// The fine-level passes of an FP32 refinement step (IrArgs).  The post pass
// leaves u itself unwritten: the iterate takes the correction directly.
template <int NU>
__global__ __launch_bounds__(FW) void k_pre_ir(Lev<float> L, float *__restrict__ uout, Wts<float> C,
                                                Lev<float> Cl, TileGeo G, const int *stop, IrArgs ir)
{
    int tid, k;
    if (!tile_work(G, tid, k)) return;
    if (stopped(stop)) return;
    __shared__ TileLds<float, false, NU> S;
    pre_tile<float, false, NU, false, true>(L, uout, C, Cl, G, tid, S, ir);
}

template <typename T, int NU>
__global__ __launch_bounds__(FW) void k_post_ir(Lev<T> L, Wts<T> C, const T *__restrict__ ec, TileGeo G,
                                                 const int *stop, IrArgs ir)
{
    int tid, k;
    if (!tile_work(G, tid, k)) return;
    if (stopped(stop)) return;
    __shared__ TileLds<T, false, NU> S;
    post_tile<T, false, NU, false, true>(L, nullptr, C, ec, G, tid, nullptr, S, ir);
}

}  // namespace bmg

namespace bmg {

// ------------------------------------ four-row steps (five-point levels)
// The same pipelines as pre_tile and post_tile with four new rows per step:
// sweep s updates the even rows e-2s and e-2s+2 (colours 0, 1) and then the
// odd rows e-2s-1 and e-2s+1 (colours 2, 3).  This is the two-row schedule of
// steps e and e+2 with their phases merged; every point sees the same
// neighbour values in the same order, so the results are the same bits, and
// each workgroup barrier now separates twice the work.  Window: rows
// e-2NU-2 .. e+3 (RW = 2NU+6), LDS rings of RW rows.
template <int R>
__device__ __forceinline__ int qslot(int row) { return (row + 64 * R) % R; }

template <typename T, int NU>
struct TileLds4 {
    static constexpr int RW = 2 * NU + 6;
    T su[RW * FW], sW[RW * FW], sx[8 * FW];
};

// five-point Gauss-Seidel update and residual from the rings (the terms of
// gs_point / residual_point in their order)
template <typename T, int R>
__device__ __forceinline__ T gs5(const T *su, const T *sW, int lane, int row, T b, T O, T S, T Sn)
{
    const int r0 = qslot<R>(row) * FW + lane;
    const int rd = qslot<R>(row - 1) * FW + lane;
    const int ru = qslot<R>(row + 1) * FW + lane;
    T s = b;
    s -= S * su[rd];
    s -= sW[r0] * su[r0 - 1];
    s -= sW[r0 + 1] * su[r0 + 1];
    s -= Sn * su[ru];
    return s / O;
}

template <typename T, int R>
__device__ __forceinline__ T res5(const T *su, const T *sW, int lane, int row, T b, T O, T S, T Sn)
{
    const int r0 = qslot<R>(row) * FW + lane;
    const int rd = qslot<R>(row - 1) * FW + lane;
    const int ru = qslot<R>(row + 1) * FW + lane;
    T s = b;
    s -= S * su[rd];
    s -= sW[r0] * su[r0 - 1];
    s -= sW[r0 + 1] * su[r0 + 1];
    s -= Sn * su[ru];
    s -= O * su[r0];
    return s;
}

template <typename T, int NU>
__device__ __forceinline__ void pre_tile4(const Lev<T> &L, T *__restrict__ uout, const Wts<T> &C,
                                          const Lev<T> &Cl, const TileGeo &G, int tid, TileLds4<T, NU> &S)
{
    constexpr int RW = 2 * NU + 6;
    T *su = S.su, *sW = S.sW, *sr = S.sx;

    const int n = L.n, ld = L.ld, lane = threadIdx.x, nc = Cl.n;
    const int useful = FW - 2 * G.hx;
    const int tx = tid % G.tiles_x, ty = tid / G.tiles_x;
    const int x0 = 1 + tx * useful;
    const int i = x0 - G.hx + lane;
    const bool col_in = i >= 0 && i <= n + 1;
    const bool col_upd = i >= 1 && i <= n && lane >= 1 && lane < FW - 1;
    const bool col_own = i >= x0 && i < x0 + useful && i <= n;
    const int y0 = 1 + ty * G.ht;
    const int y1 = min(y0 + G.ht, n + 1);
    const int es = (y0 - 2 * NU) & ~1;
    const int jlast = (y1 - 1) >> 1;
    const int elast = 2 * jlast + 2 * NU + 2;
    const int I = i >> 1;
    const bool restrictor = !(i & 1) && col_own && I >= 1 && I <= nc;

    T rO[RW], rS[RW], rB[RW];
    auto ld_row = [&](const T *a, int row) -> T {
        return (col_in && row >= 0 && row <= n + 1) ? a[(size_t)row * ld + i] : (T)0;
    };
    auto ld_w = [&](int J, T *w) {
        const bool ok = restrictor && J >= 1 && J <= nc;
        const size_t c = ok ? (size_t)J * C.ld + I : 0, cn = c + C.ld;
        w[0] = ok ? C.at(LNE, c) : (T)0;
        w[1] = ok ? C.at(LA, c) : (T)0;
        w[2] = ok ? C.at(LNW, c + 1) : (T)0;
        w[3] = ok ? C.at(LR, c) : (T)0;
        w[4] = ok ? C.at(LL, c + 1) : (T)0;
        w[5] = ok ? C.at(LSE, cn) : (T)0;
        w[6] = ok ? C.at(LB, cn) : (T)0;
        w[7] = ok ? C.at(LSW, cn + 1) : (T)0;
    };
    // window of step es without its own four rows: rows es-2NU-2 .. es-1 at
    // positions 4..RW-1 (the first shift by four aligns them)
#pragma unroll
    for (int k = 4; k < RW; ++k) {
        const int row = es - 2 * NU - 6 + k;
        su[qslot<RW>(row) * FW + lane] = ld_row(L.u, row);
        sW[qslot<RW>(row) * FW + lane] = ld_row(L.W, row);
        rO[k] = ld_row(L.O, row);
        rS[k] = ld_row(L.S, row);
        rB[k] = ld_row(L.b, row);
    }
    T pu[4], pW[4], pO[4], pS[4], pB[4], pw[16], w[16];
    auto fetch = [&](int e) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pu[q] = ld_row(L.u, e + q);
            pW[q] = ld_row(L.W, e + q);
            pO[q] = ld_row(L.O, e + q);
            pS[q] = ld_row(L.S, e + q);
            pB[q] = ld_row(L.b, e + q);
        }
        ld_w((e - 2 * NU - 2) >> 1, pw);
        ld_w(((e - 2 * NU - 2) >> 1) + 1, pw + 8);
    };
    fetch(es);

    for (int e = es; e <= elast; e += 4) {
        __syncthreads();  // the previous step is done with the slots reused below
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int sq = qslot<RW>(e + q) * FW + lane;
            su[sq] = pu[q];
            sW[sq] = pW[q];
        }
#pragma unroll
        for (int k = 0; k < RW - 4; ++k) { rO[k] = rO[k + 4]; rS[k] = rS[k + 4]; rB[k] = rB[k + 4]; }
#pragma unroll
        for (int q = 0; q < 4; ++q) { rO[RW - 4 + q] = pO[q]; rS[RW - 4 + q] = pS[q]; rB[RW - 4 + q] = pB[q]; }
#pragma unroll
        for (int q = 0; q < 16; ++q) w[q] = pw[q];
        if (e + 4 <= elast) fetch(e + 4);
        __syncthreads();
        // NU sweeps, each over colours 0,1 (two even rows) then 2,3 (two odd rows)
#pragma unroll
        for (int s = 0; s < NU; ++s) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int row = (c < 2 ? e - 2 * s : e - 2 * s - 1) + 2 * t;
                    const int k = row - (e - 2 * NU - 2);
                    if (col_upd && (i & 1) == (c & 1) && row >= 1 && row <= n)
                        su[qslot<RW>(row) * FW + lane] =
                            gs5<T, RW>(su, sW, lane, row, rB[k], rO[k], rS[k], rS[k + 1]);
                }
                __syncthreads();
            }
        }
        // the last sweep's four rows are final: write the owned ones
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = e - 2 * NU + 1 + t;
            if (col_own && row >= y0 && row < y1) uout[(size_t)row * ld + i] = su[qslot<RW>(row) * FW + lane];
        }
        // residual of rows e-2NU-1 .. e-2NU+2
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = e - 2 * NU - 1 + t;
            const int k = 1 + t;
            T r = 0;
            if (col_upd && row >= 1 && row <= n) r = res5<T, RW>(su, sW, lane, row, rB[k], rO[k], rS[k], rS[k + 1]);
            sr[(row & 7) * FW + lane] = r;
        }
        __syncthreads();
        // restriction of coarse rows (e-2NU-2)/2 and (e-2NU)/2 by the even columns
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int f = e - 2 * NU - 2 + 2 * t, J = f >> 1;
            if (restrictor && J >= 1 && J <= nc && f >= y0 && f < y1) {
                const T *wt = w + 8 * t;
                const size_t c = (size_t)J * C.ld + I;
                const T *rd = sr + ((f - 1) & 7) * FW + lane, *r0 = sr + (f & 7) * FW + lane,
                        *ru = sr + ((f + 1) & 7) * FW + lane;
                T sum = wt[0] * rd[-1];
                sum = sum + wt[1] * rd[0];
                sum = sum + wt[2] * rd[1];
                sum = sum + wt[3] * r0[-1];
                sum = sum + r0[0];
                sum = sum + wt[4] * r0[1];
                sum = sum + wt[5] * ru[-1];
                sum = sum + wt[6] * ru[0];
                sum = sum + wt[7] * ru[1];
                Cl.b[c] = sum;
                Cl.u[c] = (T)0;
            }
        }
    }
}

template <typename T, int NU>
__global__ __launch_bounds__(FW) void k_pre4(Lev<T> L, T *__restrict__ uout, Wts<T> C, Lev<T> Cl, TileGeo G,
                                              const int *stop)
{
    int tid, k;
    if (!tile_work(G, tid, k)) return;
    if (stopped(stop ? stop + k * G.kstop : stop)) return;
    L.u += k * G.ksf; L.b += k * G.ksf; uout += k * G.ksf;
    Cl.u += k * G.ksc; Cl.b += k * G.ksc;
    __shared__ TileLds4<T, NU> S;
    pre_tile4<T, NU>(L, uout, C, Cl, G, tid, S);
}

template <typename T, int NU, bool NORM>
__device__ __forceinline__ void post_tile4(const Lev<T> &L, T *__restrict__ uout, const Wts<T> &C,
                                           const T *__restrict__ ec, const TileGeo &G, int tid,
                                           double *__restrict__ part, TileLds4<T, NU> &S)
{
    static_assert(NU <= 2, "post pass supports up to two sweeps");
    constexpr int RW = 2 * NU + 6;
    T *su = S.su, *sW = S.sW, *sec = S.sx;

    const int n = L.n, ld = L.ld, lane = threadIdx.x, ldc = C.ld, nc = (n - 1) >> 1;
    const int useful = FW - 2 * G.hx;
    const int tx = tid % G.tiles_x, ty = tid / G.tiles_x;
    const int x0 = 1 + tx * useful;
    const int i = x0 - G.hx + lane;
    const bool col_in = i >= 0 && i <= n + 1;
    const bool col_upd = i >= 1 && i <= n && lane >= 1 && lane < FW - 1;
    const bool col_own = i >= x0 && i < x0 + useful && i <= n;
    const int y0 = 1 + ty * G.ht;
    const int y1 = min(y0 + G.ht, n + 1);
    const int es = (y0 - 2 * NU + 1) & ~1;
    const int elast = ((y1 + 2 * NU) + 1) & ~1;
    const int ib = (x0 - G.hx) >> 1;
    const int Ie = ib + lane;
    const bool ccol_in = lane < FW / 2 + 2 && Ie >= 0 && Ie <= nc + 1;
    const bool odd_i = i & 1;
    const int Ix = (i + 1) >> 1;

    T rO[RW], rS[RW], rB[RW];
    auto ld_row = [&](const T *a, int row) -> T {
        return (col_in && row >= 0 && row <= n + 1) ? a[(size_t)row * ld + i] : (T)0;
    };
    auto ld_crow = [&](int J) -> T {
        return (ccol_in && J >= 0 && J <= nc + 1) ? ec[(size_t)J * ldc + Ie] : (T)0;
    };
    struct IW { T w[6]; };
    // the planes this column reads for its odd row: LSW, LSE, LNW, LNE (odd
    // columns) or LB, LA (even columns); every lane issues the same six loads
    const int p2 = odd_i ? LSW : LB, p3 = odd_i ? LSE : LA;
    auto ld_iw = [&](int e) -> IW {
        IW r;
        T *w = r.w;
        const int J0 = e >> 1, J1 = J0 + 1;
        const bool ok0 = col_upd && odd_i && e >= 1 && e <= n;
        const bool ok1 = col_upd && e + 1 >= 1 && e + 1 <= n;
        const bool ok2 = ok1 && odd_i;
        const size_t c0 = ok0 ? (size_t)J0 * ldc + Ix : 0;
        const size_t c1 = ok1 ? (size_t)J1 * ldc + (odd_i ? Ix : (i >> 1)) : 0;
        w[0] = ok0 ? C.at(LL, c0) : (T)0;
        w[1] = ok0 ? C.at(LR, c0) : (T)0;
        w[2] = ok1 ? C.at(p2, c1) : (T)0;
        w[3] = ok1 ? C.at(p3, c1) : (T)0;
        w[4] = ok2 ? C.at(LNW, c1) : (T)0;
        w[5] = ok2 ? C.at(LNE, c1) : (T)0;
        return r;
    };
    // u + P e_c (the expression of post_tile's interp)
    auto interp = [&](int row, T u, const IW &iw) -> T {
        const T *w = iw.w;
        if (!col_upd || row < 1 || row > n) return u;
        T e;
        if (!(row & 1)) {
            const T *er = sec + ((row >> 1) & 3) * FW;
            if (!odd_i) e = er[(i >> 1) - ib];
            else e = w[0] * er[Ix - 1 - ib] + w[1] * er[Ix - ib];
        } else {
            const int J = (row + 1) >> 1;
            const T *es_ = sec + ((J - 1) & 3) * FW, *en = sec + (J & 3) * FW;
            if (!odd_i) {
                e = w[2] * es_[(i >> 1) - ib] + w[3] * en[(i >> 1) - ib];
            } else {
                e = w[2] * es_[Ix - 1 - ib] + w[3] * es_[Ix - ib];
                e = e + w[4] * en[Ix - 1 - ib];
                e = e + w[5] * en[Ix - ib];
            }
        }
        return u + e;
    };

    // window of step es without its own four rows: rows es-2NU-2 .. es-1,
    // interpolated, at positions 4..RW-1; their coarse rows
    // (es-2NU-2)/2 .. es/2 (at most four) fill the e_c ring
    for (int J = (es - 2 * NU - 2) >> 1; J <= (es >> 1); ++J) sec[(J & 3) * FW + lane] = ld_crow(J);
    __syncthreads();
#pragma unroll
    for (int k = 4; k < RW; k += 2) {
        const int row = es - 2 * NU - 6 + k;      // even
        const IW wk = ld_iw(row);
        su[qslot<RW>(row) * FW + lane] = interp(row, ld_row(L.u, row), wk);
        su[qslot<RW>(row + 1) * FW + lane] = interp(row + 1, ld_row(L.u, row + 1), wk);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            sW[qslot<RW>(row + t) * FW + lane] = ld_row(L.W, row + t);
            rO[k + t] = ld_row(L.O, row + t);
            rS[k + t] = ld_row(L.S, row + t);
            rB[k + t] = ld_row(L.b, row + t);
        }
    }
    T pu[4], pW[4], pO[4], pS[4], pB[4], pec[2];
    IW pw[2];
    auto fetch = [&](int e) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pu[q] = ld_row(L.u, e + q);
            pW[q] = ld_row(L.W, e + q);
            pO[q] = ld_row(L.O, e + q);
            pS[q] = ld_row(L.S, e + q);
            pB[q] = ld_row(L.b, e + q);
        }
        pec[0] = ld_crow((e >> 1) + 1);
        pec[1] = ld_crow((e >> 1) + 2);
        pw[0] = ld_iw(e);
        pw[1] = ld_iw(e + 2);
    };
    fetch(es);
    double acc = 0.0;
    for (int e = es; e <= elast; e += 4) {
        __syncthreads();
        // coarse rows e/2+1 and e/2+2 join the e_c ring
        sec[(((e >> 1) + 1) & 3) * FW + lane] = pec[0];
        sec[(((e >> 1) + 2) & 3) * FW + lane] = pec[1];
#pragma unroll
        for (int k = 0; k < RW - 4; ++k) { rO[k] = rO[k + 4]; rS[k] = rS[k + 4]; rB[k] = rB[k + 4]; }
#pragma unroll
        for (int q = 0; q < 4; ++q) { rO[RW - 4 + q] = pO[q]; rS[RW - 4 + q] = pS[q]; rB[RW - 4 + q] = pB[q]; }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int sq = qslot<RW>(e + q) * FW + lane;
            su[sq] = interp(e + q, pu[q], pw[q >> 1]);
            sW[sq] = pW[q];
        }
        if (e + 4 <= elast) fetch(e + 4);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NU; ++s) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int row = (c < 2 ? e - 2 * s : e - 2 * s - 1) + 2 * t;
                    const int k = row - (e - 2 * NU - 2);
                    if (col_upd && (i & 1) == (c & 1) && row >= 1 && row <= n)
                        su[qslot<RW>(row) * FW + lane] =
                            gs5<T, RW>(su, sW, lane, row, rB[k], rO[k], rS[k], rS[k + 1]);
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = e - 2 * NU + 1 + t;
            if (col_own && row >= y0 && row < y1) uout[(size_t)row * ld + i] = su[qslot<RW>(row) * FW + lane];
        }
        if (NORM) {
            // accurate residual of the final rows e-2NU-1 .. e-2NU+2
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = e - 2 * NU - 1 + t;
                const int k = 1 + t;
                if (col_own && row >= y0 && row < y1 && row >= 1) {
                    const int r0 = qslot<RW>(row) * FW + lane, rd = qslot<RW>(row - 1) * FW + lane,
                              ru = qslot<RW>(row + 1) * FW + lane;
                    const double a[5] = {(double)rS[k], (double)sW[r0], (double)sW[r0 + 1], (double)rS[k + 1],
                                         (double)rO[k]};
                    const double x[5] = {(double)su[rd], (double)su[r0 - 1], (double)su[r0 + 1], (double)su[ru],
                                         (double)su[r0]};
                    double sacc = rB[k], cc = 0.0, ns, se;
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        const double pr = a[q] * x[q];
                        const double pe = fma(a[q], x[q], -pr);
                        two_sum(sacc, -pr, ns, se);
                        sacc = ns;
                        cc = cc + (se - pe);
                    }
                    const double r = sacc + cc;
                    acc += r * r;
                }
            }
        }
    }
    if (NORM) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) part[tid] = acc;
    }
}

template <typename T, int NU, bool NORM>
__global__ __launch_bounds__(FW) void k_post4(Lev<T> L, T *__restrict__ uout, Wts<T> C, const T *__restrict__ ec,
                                               TileGeo G, double *__restrict__ part, const int *stop)
{
    int tid, k;
    if (!tile_work(G, tid, k)) return;
    if (stopped(stop ? stop + k * G.kstop : stop)) return;
    L.u += k * G.ksf; L.b += k * G.ksf; uout += k * G.ksf;
    ec += k * G.ksc;
    if (NORM) part += k * G.kpart;
    __shared__ TileLds4<T, NU> S;
    post_tile4<T, NU, NORM>(L, uout, C, ec, G, tid, part, S);
}

}  // namespace bmg

namespace bmg {

// ---------------------------------------------- persistent small levels
// The whole V-cycle below (and including) a small level runs in one workgroup:
// the iterates, right-hand sides and the residual of these levels stay in LDS
// (tight pitch n+2), the stencils and weights are read from global memory (they
// are a few hundred KB and stay in L2), and every phase of the cycle is
// separated by a workgroup barrier instead of a kernel launch.  On a level of
// at most 63 points per side each colour has at most 32 x 32 = SMALL_THREADS
// points, so every thread owns at most one point of each colour; it loads the
// stencil of its four points once per visit of the level and keeps it in
// registers through the sweeps and the residual (one round trip to L2 per
// visit instead of one per phase).  The arithmetic per point is the same
// expression as in the single-step kernels.
constexpr int SMALL_MAXL = 6;
constexpr int SMALL_THREADS = 1024;

template <typename T>
struct SmallH {
    int nl;                    // levels in the kernel: first .. coarsest
    Lev<T> L[SMALL_MAXL];
    Wts<T> C[SMALL_MAXL];      // C[l]: weights between L[l] and L[l+1]
    int off_u[SMALL_MAXL], off_b[SMALL_MAXL], off_r, off_z;
    BandSolve band;            // coarsest factor (one-wave band solve)
    int nu1, nu2;
    // workgroup k runs right-hand side k: the first level's u and b start
    // k*ks0 elements after the first's, its stop flag k*kstop ints after
    size_t ks0;
    int kstop;
};

constexpr int SMALL_MAX_N = 63;
constexpr int SMALL_LDS_MAX = 160 * 1024;   // LDS of one workgroup on gfx950

// The stencil rows of this thread's points, one per colour c (colour c: i odd
// if c & 1, j odd if c & 2): a[c] holds SW, S, SE (the NW entry of the point
// below-right), W, E, NW, N, NE (the SW entry of the point above-right), O in
// the order the update subtracts them; q[c] is the point's LDS index, -1 if
// the thread has no point of that colour.
template <typename T>
struct SmallPts {
    T a[4][9];
    int q[4];
};

template <typename T, bool NINE>
__device__ __forceinline__ void small_load(const Lev<T> &L, SmallPts<T> &P)
{
    const int n = L.n, p = n + 2, t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int i0 = (c & 1) ? 1 : 2, j0 = (c >> 1) ? 1 : 2;
        const int ni = (c & 1) ? (n + 1) / 2 : (n - 1) / 2, nj = (c >> 1) ? (n + 1) / 2 : (n - 1) / 2;
        const bool ok = t < ni * nj;
        const int i = ok ? i0 + 2 * (t % ni) : 1, j = ok ? j0 + 2 * (t / ni) : 1;
        const size_t g = (size_t)j * L.ld + i;
        P.q[c] = ok ? j * p + i : -1;
        T *a = P.a[c];
        a[0] = NINE && ok ? L.SW[g] : (T)0;
        a[1] = ok ? L.S[g] : (T)0;
        a[2] = NINE && ok ? L.NW[g + 1 - L.ld] : (T)0;
        a[3] = ok ? L.W[g] : (T)0;
        a[4] = ok ? L.W[g + 1] : (T)0;
        a[5] = NINE && ok ? L.NW[g] : (T)0;
        a[6] = ok ? L.S[g + L.ld] : (T)0;
        a[7] = NINE && ok ? L.SW[g + L.ld + 1] : (T)0;
        a[8] = ok ? L.O[g] : (T)1;
    }
}

// sum of the off-diagonal couplings of point q subtracted from s, in the
// order of the single-step kernels
template <typename T, bool NINE>
__device__ __forceinline__ T small_offdiag(const T *a, const T *u, int q, int p, T s)
{
    if (NINE) s -= a[0] * u[q - p - 1];
    s -= a[1] * u[q - p];
    if (NINE) s -= a[2] * u[q - p + 1];
    s -= a[3] * u[q - 1];
    s -= a[4] * u[q + 1];
    if (NINE) s -= a[5] * u[q + p - 1];
    s -= a[6] * u[q + p];
    if (NINE) s -= a[7] * u[q + p + 1];
    return s;
}

template <typename T, bool NINE>
__device__ __forceinline__ void small_relax(const SmallPts<T> &P, int p, T *u, const T *b, int sweeps)
{
    for (int s = 0; s < sweeps; ++s) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int q = P.q[c];
            if (q >= 0) u[q] = small_offdiag<T, NINE>(P.a[c], u, q, p, b[q]) / P.a[c][8];
            __syncthreads();
        }
    }
}

template <typename T, bool NINE>
__device__ __forceinline__ void small_resid(const SmallPts<T> &P, int p, const T *u, const T *b, T *r)
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int q = P.q[c];
        if (q >= 0) {
            T s = small_offdiag<T, NINE>(P.a[c], u, q, p, b[q]);
            s -= P.a[c][8] * u[q];
            r[q] = s;
        }
    }
}

// LDS elements the small sub-cycle of H needs (u and b of every level, r of
// the first), with the offsets filled in.
template <typename T>
__host__ __device__ inline int small_layout(SmallH<T> &H)
{
    int off = 0;
    for (int k = 0; k < H.nl; ++k) {
        const int p = H.L[k].n + 2;
        H.off_u[k] = off;
        off += p * p;
        H.off_b[k] = off;
        off += p * p;
    }
    H.off_r = off;
    off += (H.L[0].n + 2) * (H.L[0].n + 2);
    // FP64 scratch of the coarsest solve, 8-byte aligned
    constexpr int per = (int)(sizeof(double) / sizeof(T));
    off = (off + per - 1) / per * per;
    H.off_z = off;
    const int nL = H.L[H.nl - 1].n;
    off += band_padded(nL * nL) * per;
    return off;
}

template <typename T, bool NINE0>
__device__ void small_vcycle_body(const SmallH<T> &H, T *sm, size_t rhs_off)
{
    const int nl = H.nl, last = nl - 1;
    // fetch b of the first level, zero every iterate and the coarser b
    for (int l = 0; l < nl; ++l) {
        const int n = H.L[l].n, p = n + 2;
        T *u = sm + H.off_u[l], *b = sm + H.off_b[l];
        for (int t = threadIdx.x; t < p * p; t += blockDim.x) {
            const int i = t % p, j = t / p;
            u[t] = (T)0;
            b[t] = (l == 0 && i >= 1 && i <= n && j >= 1 && j <= n) ? H.L[0].b[rhs_off + (size_t)j * H.L[0].ld + i]
                                                                     : (T)0;
        }
    }
    T *r = sm + H.off_r;
    for (int t = threadIdx.x; t < (H.L[0].n + 2) * (H.L[0].n + 2); t += blockDim.x) r[t] = (T)0;
    __syncthreads();
    // down: relax, residual, restrict
    SmallPts<T> P;
    for (int l = 0; l < last; ++l) {
        const Lev<T> &L = H.L[l];
        T *u = sm + H.off_u[l], *b = sm + H.off_b[l];
        const int p = L.n + 2;
        if (l > 0 || NINE0) {
            small_load<T, true>(L, P);
            small_relax<T, true>(P, p, u, b, H.nu1);
            small_resid<T, true>(P, p, u, b, r);
        } else {
            small_load<T, false>(L, P);
            small_relax<T, false>(P, p, u, b, H.nu1);
            small_resid<T, false>(P, p, u, b, r);
        }
        __syncthreads();
        const int nf = L.n, pf = nf + 2, nc = H.L[l + 1].n, pc = nc + 2;
        const Wts<T> &C = H.C[l];
        T *bc = sm + H.off_b[l + 1];
        for (int t = threadIdx.x; t < nc * nc; t += blockDim.x) {
            const int I = 1 + t % nc, J = 1 + t / nc;
            const size_t c = (size_t)J * C.ld + I, cn = c + C.ld;
            const int f = (2 * J) * pf + 2 * I;
            T s = C.at(LNE, c) * r[f - pf - 1];
            s = s + C.at(LA, c) * r[f - pf];
            s = s + C.at(LNW, c + 1) * r[f - pf + 1];
            s = s + C.at(LR, c) * r[f - 1];
            s = s + r[f];
            s = s + C.at(LL, c + 1) * r[f + 1];
            s = s + C.at(LSE, cn) * r[f + pf - 1];
            s = s + C.at(LB, cn) * r[f + pf];
            s = s + C.at(LSW, cn + 1) * r[f + pf + 1];
            bc[J * pc + I] = s;
        }
        __syncthreads();
    }
    // coarsest level: the band LDL^T solve in FP64 by the first wave
    if (threadIdx.x < 64) {
        const int nc = H.L[last].n, pc = nc + 2;
        const T *b = sm + H.off_b[last];
        T *u = sm + H.off_u[last];
        band_solve_direct(
            H.band, [&](int k) -> double { return (double)b[(k / nc + 1) * pc + k % nc + 1]; },
            [&](int k, double x) { u[(k / nc + 1) * pc + k % nc + 1] = (T)x; },
            reinterpret_cast<double *>(sm + H.off_z));
    }
    __syncthreads();
    // up: interpolate and correct, relax
    for (int l = last - 1; l >= 0; --l) {
        const Lev<T> &L = H.L[l];
        T *u = sm + H.off_u[l], *b = sm + H.off_b[l];
        const T *ec = sm + H.off_u[l + 1];
        const int n = L.n, p = n + 2, pc = H.L[l + 1].n + 2;
        const Wts<T> &C = H.C[l];
        const bool nine = (l > 0) || NINE0;
        // the sweeps' stencil is requested before the interpolation runs
        if (nine) small_load<T, true>(L, P); else small_load<T, false>(L, P);
        for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
            const int i = 1 + t % n, j = 1 + t / n;
            T e;
            if (!(i & 1) && !(j & 1)) {
                e = ec[(j >> 1) * pc + (i >> 1)];
            } else if ((i & 1) && !(j & 1)) {
                const int I = (i + 1) >> 1, J = j >> 1;
                const size_t c = (size_t)J * C.ld + I;
                e = C.at(LL, c) * ec[J * pc + I - 1] + C.at(LR, c) * ec[J * pc + I];
            } else if (!(i & 1)) {
                const int I = i >> 1, J = (j + 1) >> 1;
                const size_t c = (size_t)J * C.ld + I;
                e = C.at(LB, c) * ec[(J - 1) * pc + I] + C.at(LA, c) * ec[J * pc + I];
            } else {
                const int I = (i + 1) >> 1, J = (j + 1) >> 1;
                const size_t c = (size_t)J * C.ld + I;
                e = C.at(LSW, c) * ec[(J - 1) * pc + I - 1] + C.at(LSE, c) * ec[(J - 1) * pc + I];
                e = e + C.at(LNW, c) * ec[J * pc + I - 1];
                e = e + C.at(LNE, c) * ec[J * pc + I];
            }
            u[j * p + i] = u[j * p + i] + e;
        }
        __syncthreads();
        if (nine) small_relax<T, true>(P, p, u, b, H.nu2); else small_relax<T, false>(P, p, u, b, H.nu2);
    }
    // the first level's iterate back to global memory
    {
        const Lev<T> &L = H.L[0];
        const int n = L.n, p = n + 2;
        const T *u = sm + H.off_u[0];
        for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
            const int i = 1 + t % n, j = 1 + t / n;
            L.u[rhs_off + (size_t)j * L.ld + i] = u[j * p + i];
        }
    }
}

template <typename T, bool NINE0>
__global__ __launch_bounds__(SMALL_THREADS) void k_small_vcycle(SmallH<T> H, const int *stop)
{
    const int k = blockIdx.x;
    if (stopped(stop ? stop + k * H.kstop : stop)) return;
    extern __shared__ unsigned char smem_raw[];
    small_vcycle_body<T, NINE0>(H, reinterpret_cast<T *>(smem_raw), k * H.ks0);
}

}  // namespace bmg
