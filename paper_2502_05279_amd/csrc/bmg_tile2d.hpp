// Passes of the small nine-point levels in square tiles: one workgroup loads a
// tile of the level with its halo into LDS at once (u and b; each thread keeps
// the nine stencil entries of its points in registers), runs every colour
// phase of the sweeps there with a workgroup barrier between phases, and
// writes the owned points.  On levels of a few hundred points per side the
// row pipeline of the streaming passes walks a chain of dependent steps per
// tile, each waiting on its own loads; here a pass waits on memory once.
// The halo makes every owned output exact: the outermost ring of the tile is
// never updated and each colour phase can carry its staleness one point
// inward, so nu sweeps (4 nu phases) plus the residual and the restriction
// need 4 nu + 2 points (the post pass, without residual, 4 nu).  Every point's
// expressions are those of gs_point, residual_point, interp_point and
// k_restrict, so the results are those of the separate kernels to the bit.
#pragma once

#include "bmg_kernels.hpp"

namespace bmg {

constexpr int T2D = 32;            // owned fine points per side of a tile
constexpr int T2D_THREADS = 1024;
constexpr int T2D_MAX_N = 511;     // levels this runs on (nine-point, one right-hand side)

__host__ __device__ constexpr int t2d_side(int halo) { return T2D + 2 * halo; }
__host__ __device__ constexpr int t2d_slots(int halo) { return (t2d_side(halo) * t2d_side(halo) + T2D_THREADS - 1) / T2D_THREADS; }

template <typename T, int HALO>
struct T2dPts {
    static constexpr int S = t2d_side(HALO), SL = t2d_slots(HALO);
    T a[SL][9];       // SW, S, SE, W, O, E, NW, N, NE of each point
    int gi[SL], gj[SL];
};

// The tile's point k (k = threadIdx.x + s * T2D_THREADS) at level indices
// (gi, gj); nine entries of interior points, zeros elsewhere.
template <typename T, int HALO>
__device__ __forceinline__ void t2d_load(const Lev<T> &L, int x0, int y0, T *su, T *sb, T2dPts<T, HALO> &P)
{
    constexpr int S = T2dPts<T, HALO>::S;
    const size_t ld = L.ld;
#pragma unroll
    for (int s = 0; s < T2dPts<T, HALO>::SL; ++s) {
        const int k = threadIdx.x + s * T2D_THREADS;
        const int li = k % S, lj = k / S;
        const int gi = x0 - HALO + li, gj = y0 - HALO + lj;
        P.gi[s] = gi;
        P.gj[s] = gj;
        const bool in = k < S * S;
        const bool any = in && gi >= 0 && gi <= L.n + 1 && gj >= 0 && gj <= L.n + 1;
        const bool inner = in && gi >= 1 && gi <= L.n && gj >= 1 && gj <= L.n;
        const size_t p = any ? (size_t)gj * ld + gi : 0;
        if (in) {
            su[k] = any ? L.u[p] : (T)0;
            sb[k] = any ? L.b[p] : (T)0;
        }
        T *a = P.a[s];
        a[0] = inner ? L.SW[p] : (T)0;
        a[1] = inner ? L.S[p] : (T)0;
        a[2] = inner ? L.NW[p + 1 - ld] : (T)0;
        a[3] = inner ? L.W[p] : (T)0;
        a[4] = inner ? L.O[p] : (T)1;
        a[5] = inner ? L.W[p + 1] : (T)0;
        a[6] = inner ? L.NW[p] : (T)0;
        a[7] = inner ? L.S[p + ld] : (T)0;
        a[8] = inner ? L.SW[p + ld + 1] : (T)0;
    }
}

// b minus the eight couplings, in gs_point's order.
template <typename T, int S>
__device__ __forceinline__ T t2d_offdiag(const T *a, const T *su, int k, T s)
{
    s -= a[0] * su[k - S - 1];
    s -= a[1] * su[k - S];
    s -= a[2] * su[k - S + 1];
    s -= a[3] * su[k - 1];
    s -= a[5] * su[k + 1];
    s -= a[6] * su[k + S - 1];
    s -= a[7] * su[k + S];
    s -= a[8] * su[k + S + 1];
    return s;
}

// NU four-colour sweeps on the tile's interior points away from its outer ring.
template <typename T, int HALO, int NU>
__device__ __forceinline__ void t2d_sweeps(const Lev<T> &L, T *su, const T *sb, const T2dPts<T, HALO> &P)
{
    constexpr int S = T2dPts<T, HALO>::S;
    for (int sw = 0; sw < NU; ++sw) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int s = 0; s < T2dPts<T, HALO>::SL; ++s) {
                const int k = threadIdx.x + s * T2D_THREADS;
                const int li = k % S, lj = k / S, gi = P.gi[s], gj = P.gj[s];
                if (k < S * S && li >= 1 && li <= S - 2 && lj >= 1 && lj <= S - 2 && gi >= 1 && gi <= L.n &&
                    gj >= 1 && gj <= L.n && (gi & 1) + 2 * (gj & 1) == c)
                    su[k] = t2d_offdiag<T, S>(P.a[s], su, k, sb[k]) / P.a[s][4];
            }
            __syncthreads();
        }
    }
}

// Pre pass: NU sweeps, residual on the owned points and one ring around them,
// restriction of the owned coarse points (b_c, u_c = 0), u of the owned
// points to uout.
template <typename T, int NU>
__global__ __launch_bounds__(T2D_THREADS) void k_pre2d(Lev<T> L, T *__restrict__ uout, Wts<T> C, Lev<T> Cl,
                                                      const int *stop)
{
    if (stopped(stop)) return;
    constexpr int HALO = 4 * NU + 2, S = t2d_side(HALO), R = T2D + 2;
    __shared__ T su[S * S], sb[S * S], sr[R * R];
    const int x0 = 1 + T2D * blockIdx.x, y0 = 1 + T2D * blockIdx.y;
    T2dPts<T, HALO> P;
    t2d_load<T, HALO>(L, x0, y0, su, sb, P);
    __syncthreads();
    t2d_sweeps<T, HALO, NU>(L, su, sb, P);
    // residual on [x0-1, x0+T2D] x [y0-1, y0+T2D] (zero outside the interior)
#pragma unroll
    for (int s = 0; s < T2dPts<T, HALO>::SL; ++s) {
        const int k = threadIdx.x + s * T2D_THREADS;
        const int li = k % S, lj = k / S, gi = P.gi[s], gj = P.gj[s];
        const int ri = li - (HALO - 1), rj = lj - (HALO - 1);
        if (k < S * S && ri >= 0 && ri < R && rj >= 0 && rj < R) {
            T r = (T)0;
            if (gi >= 1 && gi <= L.n && gj >= 1 && gj <= L.n) {
                r = t2d_offdiag<T, S>(P.a[s], su, k, sb[k]);
                r -= P.a[s][4] * su[k];
            }
            sr[rj * R + ri] = r;
        }
        // the owned points' new values
        if (k < S * S && li >= HALO && li < HALO + T2D && lj >= HALO && lj < HALO + T2D && gi <= L.n && gj <= L.n)
            uout[(size_t)gj * L.ld + gi] = su[k];
    }
    __syncthreads();
    // restriction: coarse (I, J) with (2I, 2J) owned, in k_restrict's order
    const int nco = T2D / 2;
    if (threadIdx.x < nco * nco) {
        const int I = (x0 + 1) / 2 + threadIdx.x % nco, J = (y0 + 1) / 2 + threadIdx.x / nco;
        if (I <= Cl.n && J <= Cl.n) {
            const size_t c = (size_t)J * C.ld + I;
            const size_t cn = c + C.ld;
            const int fi = 2 * I - (x0 - 1), fj = 2 * J - (y0 - 1);   // (2I, 2J) in the residual tile
            const T *rd = sr + (fj - 1) * R + fi, *r0 = sr + fj * R + fi, *ru = sr + (fj + 1) * R + fi;
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

// Post pass: u += P e_c on the tile, NU sweeps, u of the owned points to uout.
template <typename T, int NU>
__global__ __launch_bounds__(T2D_THREADS) void k_post2d(Lev<T> L, T *__restrict__ uout, Wts<T> C,
                                                       const T *__restrict__ ec, const int *stop)
{
    if (stopped(stop)) return;
    constexpr int HALO = 4 * NU, S = t2d_side(HALO);
    __shared__ T su[S * S], sb[S * S];
    const int x0 = 1 + T2D * blockIdx.x, y0 = 1 + T2D * blockIdx.y;
    T2dPts<T, HALO> P;
    t2d_load<T, HALO>(L, x0, y0, su, sb, P);
#pragma unroll
    for (int s = 0; s < T2dPts<T, HALO>::SL; ++s) {
        const int k = threadIdx.x + s * T2D_THREADS, gi = P.gi[s], gj = P.gj[s];
        if (k < S * S && gi >= 1 && gi <= L.n && gj >= 1 && gj <= L.n) su[k] = su[k] + interp_point<T>(C, ec, gi, gj);
    }
    __syncthreads();
    t2d_sweeps<T, HALO, NU>(L, su, sb, P);
#pragma unroll
    for (int s = 0; s < T2dPts<T, HALO>::SL; ++s) {
        const int k = threadIdx.x + s * T2D_THREADS;
        const int li = k % S, lj = k / S, gi = P.gi[s], gj = P.gj[s];
        if (k < S * S && li >= HALO && li < HALO + T2D && lj >= HALO && lj < HALO + T2D && gi <= L.n && gj <= L.n)
            uout[(size_t)gj * L.ld + gi] = su[k];
    }
}

}  // namespace bmg
