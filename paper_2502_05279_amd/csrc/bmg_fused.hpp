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
__device__ __forceinline__ int slot(int row) { return (row + 64 * R) & (R - 1); }

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
};

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
// tile; u_c = 0 there.  Window: rows e-2NU-2 .. e+1 (RW rows) at step e.
template <typename T, bool NINE, int NU>
__global__ __launch_bounds__(FW) void k_pre(Lev<T> L, T *__restrict__ uout, Wts<T> C, Lev<T> Cl,
                                             TileGeo G, const int *stop)
{
    if (stopped(stop)) return;
    const int tid = tile_id(G.ntiles);
    if (tid < 0) return;
    constexpr int RW = 2 * NU + 4;                 // window rows
    constexpr int RU = RW <= 8 ? 8 : 16;           // LDS ring rows (power of two)
    __shared__ T su[RU * FW], sW[RU * FW], sr[4 * FW];
    __shared__ T sSW[NINE ? RU * FW : 1], sNW[NINE ? RU * FW : 1];

    const int n = L.n, ld = L.ld, lane = threadIdx.x;
    const int useful = FW - 2 * G.hx;
    const int tx = tid % G.tiles_x, ty = tid / G.tiles_x;
    const int x0 = 1 + tx * useful;                // first owned column
    const int i = x0 - G.hx + lane;                // this lane's column
    const bool col_in = i >= 0 && i <= n + 1;
    const bool col_upd = i >= 1 && i <= n && lane >= 1 && lane < FW - 1;
    const bool col_own = i >= x0 && i < x0 + useful && i <= n;
    const int y0 = 1 + ty * G.ht;                  // owned rows [y0, y1)
    const int y1 = min(y0 + G.ht, n + 1);
    const int es = (y0 - 2 * NU) & ~1;             // first even row of sweep 0: the
                                                   // warm-up below y0 that makes the
                                                   // owned rows and coarse rows exact
    const int jlast = (y1 - 1) >> 1;               // last owned coarse row
    const int elast = 2 * jlast + 2 * NU + 2;      // step that restricts it

    // register windows: k <-> row e - 2NU - 2 + k
    T rO[RW], rS[RW], rB[RW];
    auto ld_row = [&](const T *a, int row) -> T {
        return (col_in && row >= 0 && row <= n + 1) ? a[(size_t)row * ld + i] : (T)0;
    };
    // initial window for step es: rows es-2NU-2 .. es-1 (the loop loads es, es+1)
#pragma unroll
    for (int k = 0; k < RW - 2; ++k) {
        const int row = es - 2 * NU - 2 + k;
        su[slot<RU>(row) * FW + lane] = ld_row(L.u, row);
        sW[slot<RU>(row) * FW + lane] = ld_row(L.W, row);
        if (NINE) {
            sSW[slot<RU>(row) * FW + lane] = ld_row(L.SW, row);
            sNW[slot<RU>(row) * FW + lane] = ld_row(L.NW, row);
        }
        rO[k] = ld_row(L.O, row);
        rS[k] = ld_row(L.S, row);
        rB[k] = ld_row(L.b, row);
    }
    // prefetch for the first step
    T pu0 = ld_row(L.u, es), pu1 = ld_row(L.u, es + 1);
    T pW0 = ld_row(L.W, es), pW1 = ld_row(L.W, es + 1);
    T pO0 = ld_row(L.O, es), pO1 = ld_row(L.O, es + 1);
    T pS0 = ld_row(L.S, es), pS1 = ld_row(L.S, es + 1);
    T pB0 = ld_row(L.b, es), pB1 = ld_row(L.b, es + 1);
    T pSW0 = 0, pSW1 = 0, pNW0 = 0, pNW1 = 0;
    if (NINE) {
        pSW0 = ld_row(L.SW, es); pSW1 = ld_row(L.SW, es + 1);
        pNW0 = ld_row(L.NW, es); pNW1 = ld_row(L.NW, es + 1);
    }

    for (int e = es; e <= elast; e += 2) {
        __syncthreads();  // the previous step is done with the slots reused below
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
        }
        // prefetch the next step's rows
        if (e + 2 <= elast) {
            pu0 = ld_row(L.u, e + 2); pu1 = ld_row(L.u, e + 3);
            pW0 = ld_row(L.W, e + 2); pW1 = ld_row(L.W, e + 3);
            pO0 = ld_row(L.O, e + 2); pO1 = ld_row(L.O, e + 3);
            pS0 = ld_row(L.S, e + 2); pS1 = ld_row(L.S, e + 3);
            pB0 = ld_row(L.b, e + 2); pB1 = ld_row(L.b, e + 3);
            if (NINE) {
                pSW0 = ld_row(L.SW, e + 2); pSW1 = ld_row(L.SW, e + 3);
                pNW0 = ld_row(L.NW, e + 2); pNW1 = ld_row(L.NW, e + 3);
            }
        }
        __syncthreads();
        // NU sweeps, each over colours 0,1 (even row) then 2,3 (odd row)
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
        // the last sweep's two rows are final: write the owned ones
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int row = e - 2 * NU + 2 - t;
            if (col_own && row >= y0 && row < y1)
                uout[(size_t)row * ld + i] = su[slot<RU>(row) * FW + lane];
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
        __syncthreads();
        // restriction of coarse row J = (e - 2NU - 2) / 2 by the even columns
        {
            const int f = e - 2 * NU - 2, J = f >> 1, I = i >> 1;
            if (!(i & 1) && col_own && J >= 1 && J <= Cl.n && f >= y0 && f < y1 && I >= 1 && I <= Cl.n) {
                const size_t c = (size_t)J * C.ld + I, cn = c + C.ld;
                const T *rd = sr + ((f - 1) & 3) * FW + lane, *r0 = sr + (f & 3) * FW + lane,
                        *ru = sr + ((f + 1) & 3) * FW + lane;
                T s = C.at(LNE, c) * rd[-1];
                s = s + C.at(LA, c) * rd[0];
                s = s + C.at(LNW, c + 1) * rd[1];
                s = s + C.at(LR, c) * r0[-1];
                s = s + r0[0];
                s = s + C.at(LL, c + 1) * r0[1];
                s = s + C.at(LSE, cn) * ru[-1];
                s = s + C.at(LB, cn) * ru[0];
                s = s + C.at(LSW, cn + 1) * ru[1];
                Cl.b[c] = s;
                Cl.u[c] = (T)0;
            }
        }
    }
}

// ---------------------------------------------------------- post pass
// u_out = GS^NU(u_in + P e_c).  With NORM (FP64 fine level) also the
// per-tile sum of squares of the accurate residual b - A u_out over the owned
// points into part[tile].  Window: rows e-2NU-2 .. e+1 at step e.
template <typename T, bool NINE, int NU, bool NORM>
__global__ __launch_bounds__(FW) void k_post(Lev<T> L, T *__restrict__ uout, Wts<T> C, const T *__restrict__ ec,
                                              TileGeo G, double *__restrict__ part, const int *stop)
{
    if (stopped(stop)) return;
    const int tid = tile_id(G.ntiles);
    if (tid < 0) return;
    constexpr int RW = 2 * NU + 4;
    constexpr int RU = RW <= 8 ? 8 : 16;
    __shared__ T su[RU * FW], sW[RU * FW], sec[4 * FW];
    __shared__ T sSW[NINE ? RU * FW : 1], sNW[NINE ? RU * FW : 1];

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

    T rO[RW], rS[RW], rB[RW];
    auto ld_row = [&](const T *a, int row) -> T {
        return (col_in && row >= 0 && row <= n + 1) ? a[(size_t)row * ld + i] : (T)0;
    };
    auto ld_crow = [&](int J) -> T {
        return (ccol_in && J >= 0 && J <= nc + 1) ? ec[(size_t)J * ldc + Ie] : (T)0;
    };
    // u + P e_c at (i, row), e_c rows of the LDS ring
    auto interp = [&](int row, T u) -> T {
        if (!col_upd || row < 1 || row > n) return u;
        T e;
        const int li = lane;  // fine column i <-> coarse column (i >> 1) - ib
        if (!(i & 1) && !(row & 1)) {
            e = sec[((row >> 1) & 3) * FW + (i >> 1) - ib];
        } else if ((i & 1) && !(row & 1)) {
            const int J = row >> 1, I = (i + 1) >> 1;
            const size_t c = (size_t)J * ldc + I;
            const T *er = sec + (J & 3) * FW + (I - ib);
            e = C.at(LL, c) * er[-1] + C.at(LR, c) * er[0];
        } else if (!(i & 1)) {
            const int J = (row + 1) >> 1, I = i >> 1;
            const size_t c = (size_t)J * ldc + I;
            e = C.at(LB, c) * sec[((J - 1) & 3) * FW + (I - ib)] + C.at(LA, c) * sec[(J & 3) * FW + (I - ib)];
        } else {
            const int J = (row + 1) >> 1, I = (i + 1) >> 1;
            const size_t c = (size_t)J * ldc + I;
            const T *es_ = sec + ((J - 1) & 3) * FW + (I - ib), *en = sec + (J & 3) * FW + (I - ib);
            e = C.at(LSW, c) * es_[-1] + C.at(LSE, c) * es_[0];
            e = e + C.at(LNW, c) * en[-1];
            e = e + C.at(LNE, c) * en[0];
        }
        (void)li;
        return u + e;
    };

    // initial window rows es-2NU-2 .. es-1: interpolated u; their coarse rows
    // are (es-2NU-2)/2 .. es/2 (NU + 2 <= 4 rows, the e_c ring)
    static_assert(NU <= 2, "post pass supports up to two sweeps");
    for (int J = (es - 2 * NU - 2) >> 1; J <= (es >> 1); ++J) sec[(J & 3) * FW + lane] = ld_crow(J);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RW - 2; ++k) {
        const int row = es - 2 * NU - 2 + k;
        su[slot<RU>(row) * FW + lane] = interp(row, ld_row(L.u, row));
        sW[slot<RU>(row) * FW + lane] = ld_row(L.W, row);
        if (NINE) {
            sSW[slot<RU>(row) * FW + lane] = ld_row(L.SW, row);
            sNW[slot<RU>(row) * FW + lane] = ld_row(L.NW, row);
        }
        rO[k] = ld_row(L.O, row);
        rS[k] = ld_row(L.S, row);
        rB[k] = ld_row(L.b, row);
    }
    double acc = 0.0;
    for (int e = es; e <= elast; e += 2) {
        __syncthreads();
        // coarse row e/2 + 1 joins the e_c ring (rows e/2 and e/2 + 1 are used)
        sec[(((e >> 1) + 1) & 3) * FW + lane] = ld_crow((e >> 1) + 1);
        const T u0 = ld_row(L.u, e), u1 = ld_row(L.u, e + 1);
        const T w0 = ld_row(L.W, e), w1 = ld_row(L.W, e + 1);
        T sw0 = 0, sw1 = 0, nw0 = 0, nw1 = 0;
        if (NINE) { sw0 = ld_row(L.SW, e); sw1 = ld_row(L.SW, e + 1); nw0 = ld_row(L.NW, e); nw1 = ld_row(L.NW, e + 1); }
#pragma unroll
        for (int k = 0; k < RW - 2; ++k) { rO[k] = rO[k + 2]; rS[k] = rS[k + 2]; rB[k] = rB[k + 2]; }
        rO[RW - 2] = ld_row(L.O, e); rO[RW - 1] = ld_row(L.O, e + 1);
        rS[RW - 2] = ld_row(L.S, e); rS[RW - 1] = ld_row(L.S, e + 1);
        rB[RW - 2] = ld_row(L.b, e); rB[RW - 1] = ld_row(L.b, e + 1);
        __syncthreads();
        {
            const int s0 = slot<RU>(e) * FW + lane, s1 = slot<RU>(e + 1) * FW + lane;
            su[s0] = interp(e, u0);
            su[s1] = interp(e + 1, u1);
            sW[s0] = w0; sW[s1] = w1;
            if (NINE) { sSW[s0] = sw0; sSW[s1] = sw1; sNW[s0] = nw0; sNW[s1] = nw1; }
        }
        __syncthreads();
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
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int row = e - 2 * NU + 2 - t;
            if (col_own && row >= y0 && row < y1)
                uout[(size_t)row * ld + i] = su[slot<RU>(row) * FW + lane];
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
        acc = block_sum(acc);
        if (threadIdx.x == 0) part[tid] = acc;
    }
}

}  // namespace bmg
