// Learned interpolation on gfx950: a three-layer 3x3 convolutional network
// that maps the normalised fine stencil to the eight interpolation-weight
// planes, its backward pass, Adam, the two-grid training objective with its
// adjoint, and the probe-and-fallback solve.  The convolutions are implicit
// GEMMs on the matrix cores (v_mfma_f32_16x16x16_bf16: bfloat16 operands,
// FP32 accumulation); activations are stored bfloat16 with the channels of a
// point contiguous, so one lane's four consecutive channels are one 8-byte
// load or store.
#include "bmg_internal.hpp"

#include <cmath>
#include <cstring>

using namespace bmgi;

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

// flat parameter vector
constexpr int NP = BMG_NET_PARAMS;
constexpr int OW1 = 0, OB1 = OW1 + 9 * 9 * 32, OW2 = OB1 + 32, OB2 = OW2 + 9 * 32 * 32, OW3 = OB2 + 32,
              OB3 = OW3 + 9 * 32 * 8;
static_assert(OB3 + 8 == NP, "parameter layout");

// packed MFMA A-operands: [tap][k-block][m-block][64 lanes] x 4 bfloat16
constexpr int PK1 = 9 * 1 * 2 * 64;   // conv1 forward: M = 32 out, K = 16 in (9 used)
constexpr int PK2 = 9 * 2 * 2 * 64;   // conv2 forward: M = 32, K = 32
constexpr int PK3 = 9 * 2 * 1 * 64;   // conv3 forward: M = 16 (8 used), K = 32
constexpr int PK2T = 9 * 2 * 2 * 64;  // conv2 backward (transposed): M = 32 in, K = 32 out
constexpr int PK3T = 9 * 1 * 2 * 64;  // conv3 backward: M = 32 in, K = 16 out (8 used)
constexpr int PKO1 = 0, PKO2 = PKO1 + PK1, PKO3 = PKO2 + PK2, PKO2T = PKO3 + PK3, PKO3T = PKO2T + PK2T,
              PK_TOTAL = PKO3T + PK3T;

constexpr int WG_WAVES = 512;                       // waves of a weight-gradient launch
constexpr int WG_SLOT = 9 * 32 * 32 + 32;           // partial of one wave (largest layer)

__device__ __forceinline__ bf16_t bf16_rne(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(bf16_t h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ uint2 pack4(bf16_t a, bf16_t b, bf16_t c, bf16_t d)
{
    return make_uint2((unsigned)a | ((unsigned)b << 16), (unsigned)c | ((unsigned)d << 16));
}

// ------------------------------------------------------------ weight packing
// One thread per packed bfloat16.  Forward operands hold A[m = out][k = in],
// transposed ones A[m = in][k = out]; lane l of a 16x16 block holds row l%16,
// columns 4(l/16)..4(l/16)+3.
__device__ bf16_t packed_value(const float *__restrict__ W, int cin, int cout, int KB, int MB, bool tr, int idx)
{
    const int e = idx & 3, lane = (idx >> 2) & 63;
    int rest = idx >> 8;
    const int mb = rest % MB;
    rest /= MB;
    const int kb = rest % KB;
    const int t = rest / KB;
    const int m = mb * 16 + (lane & 15), k = kb * 16 + 4 * (lane >> 4) + e;
    const int ci = tr ? m : k, co = tr ? k : m;
    if (ci >= cin || co >= cout) return 0;
    return bf16_rne(W[((size_t)t * cin + ci) * cout + co]);
}

static __global__ void k_pack_weights(const float *__restrict__ P, bf16_t *__restrict__ out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= PK_TOTAL * 4) return;
    const int u = g >> 2;   // uint2 index
    int idx;
    bf16_t v;
    if (u < PKO2) { idx = g - PKO1 * 4; v = packed_value(P + OW1, 9, 32, 1, 2, false, idx); }
    else if (u < PKO3) { idx = g - PKO2 * 4; v = packed_value(P + OW2, 32, 32, 2, 2, false, idx); }
    else if (u < PKO2T) { idx = g - PKO3 * 4; v = packed_value(P + OW3, 32, 8, 2, 1, false, idx); }
    else if (u < PKO3T) { idx = g - PKO2T * 4; v = packed_value(P + OW2, 32, 32, 2, 2, true, idx); }
    else { idx = g - PKO3T * 4; v = packed_value(P + OW3, 32, 8, 1, 2, true, idx); }
    out[g] = v;
}

// ------------------------------------------------------------------ features
// X(p) = bf16(fl32(a_c(p) / O(p))) for the nine coefficients SW..NE of every
// interior point, channels 9..15 and the ring zero.  One thread per point of
// the padded grid, 32 bytes each.
static __global__ void k_net_features(Lev<double> L, bool nine, bf16_t *__restrict__ X)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int n = L.n, side = n + 2;
    if (i >= side || j >= side) return;
    bf16_t v[16] = {};
    if (i >= 1 && i <= n && j >= 1 && j <= n) {
        const size_t ld = L.ld, p = (size_t)j * ld + i;
        double a[9];
        a[0] = nine ? L.SW[p] : 0.0;
        a[1] = L.S[p];
        a[2] = nine ? L.NW[p + 1 - ld] : 0.0;
        a[3] = L.W[p];
        a[4] = L.O[p];
        a[5] = L.W[p + 1];
        a[6] = nine ? L.NW[p] : 0.0;
        a[7] = L.S[p + ld];
        a[8] = nine ? L.SW[p + ld + 1] : 0.0;
        const double o = a[4];
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c] = bf16_rne((float)(a[c] / o));
    }
    uint2 *dst = reinterpret_cast<uint2 *>(X + ((size_t)j * side + i) * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = pack4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// ------------------------------------------------------------- convolutions
// Implicit-GEMM 3x3 convolution, D[out channel][point] = sum over taps and
// input channels of W * input, groups of 16 output points of one grid row per wave.
// MODE 0: input centre = output point (stride 1); 1: centre = 2 x output point
// (stride 2); 2: transposed stride 1 (input at point - tap, backward of a
// stride-1 layer); 3: transposed stride 2 (input at (point - tap) / 2 where
// both coordinates are even).  Epilogues: EP_RELU stores bf16(max(z, 0));
// EP_MASK stores bf16(z) where the mask activation is non-zero, else 0;
// EP_OUT stores the eight FP32 outputs per point (the corrections that
// k_net_apply turns into weight planes).  Points of the output domain outside
// the valid region are written as zeros.
enum { EP_RELU = 0, EP_MASK = 1, EP_OUT = 2 };

struct ConvArgs {
    const bf16_t *in;
    int in_side;                 // points per row of the input grid
    const uint2 *w;              // packed A operands of this layer
    const float *bias;           // nullptr: none
    int cout;                    // real output channels
    int lo, hi;                  // output domain [lo, hi]^2
    int vlo, vhi;                // valid region [vlo, vhi]^2
    bf16_t *out;                 // EP_RELU / EP_MASK
    int out_side;
    const bf16_t *mask;          // EP_MASK: activation (COUTP channels per point)
    int mask_side;
    float *yout;                 // EP_OUT: 8 values per point, out_side points per row
};

// Each wave keeps the layer's A operands (all taps and channel blocks) in
// registers and computes CONV_GROUPS groups of 16 consecutive output points
// of its row with them, so the weights are read once per wave instead of once
// per group; every group's products are accumulated in the same order as
// before (taps, input blocks, output blocks).
constexpr int CONV_GROUPS = 4;
template <int CINP, int COUTP, int MODE, int EP>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a)
{
    constexpr int KB = CINP / 16, MB = COUTP / 16, NA = 9 * KB * MB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = a.lo + blockIdx.y;
    const int ibase = a.lo + (blockIdx.x * 4 + wave) * 16 * CONV_GROUPS;
    if (ibase > a.hi) return;   // whole wave past the row end; no barriers below
    const int kq = 4 * (lane >> 4);
    const bool row_valid = j >= a.vlo && j <= a.vhi;

    bf16x4 wr[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const uint2 wv = a.w[q * 64 + lane];
        wr[q][0] = (short)(wv.x & 0xffff);
        wr[q][1] = (short)(wv.x >> 16);
        wr[q][2] = (short)(wv.y & 0xffff);
        wr[q][3] = (short)(wv.y >> 16);
    }
    float bias[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = mb * 16 + kq + e;
            bias[mb][e] = (a.bias && co < a.cout) ? a.bias[co] : 0.0f;
        }

    // the input fragments of a group (tap t, channel block kb); those of the
    // next group are requested before this group's products, so a wave waits
    // for its inputs once rather than once per group
    auto load_group = [&](int g, bf16x4 (&in)[9][KB]) {
        const int pi = ibase + 16 * g + (lane & 15);
        const bool valid = row_valid && pi <= a.hi && pi >= a.vlo && pi <= a.vhi;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dx = t % 3 - 1, dy = t / 3 - 1;
            bool ok = valid;
            int sx, sy;
            if (MODE == 0) { sx = pi + dx; sy = j + dy; }
            else if (MODE == 1) { sx = 2 * pi + dx; sy = 2 * j + dy; }
            else if (MODE == 2) { sx = pi - dx; sy = j - dy; }
            else {
                ok = ok && (((pi - dx) & 1) == 0) && (((j - dy) & 1) == 0);
                sx = (pi - dx) >> 1;
                sy = (j - dy) >> 1;
            }
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                bf16x4 v = {0, 0, 0, 0};
                if (ok) v = *reinterpret_cast<const bf16x4 *>(a.in + ((size_t)sy * a.in_side + sx) * CINP + kb * 16 + kq);
                in[t][kb] = v;
            }
        }
    };
    bf16x4 cur[9][KB], nxt[9][KB];
    load_group(0, cur);
#pragma unroll
    for (int g = 0; g < CONV_GROUPS; ++g) {
        const int i0 = ibase + 16 * g;
        if (i0 > a.hi) break;
        if (g + 1 < CONV_GROUPS && i0 + 16 <= a.hi) load_group(g + 1, nxt);
        const int pi = i0 + (lane & 15);
        const bool in_dom = pi <= a.hi;
        const bool valid = in_dom && row_valid && pi >= a.vlo && pi <= a.vhi;
        f32x4 acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[mb][e] = bias[mb][e];
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wr[(t * KB + kb) * MB + mb], cur[t][kb],
                                                                       acc[mb], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) cur[t][kb] = nxt[t][kb];
        if (!in_dom) continue;
        if (EP == EP_OUT) {
            if (kq < 8) {
                float4 v;
                v.x = valid ? acc[0][0] : 0.0f;
                v.y = valid ? acc[0][1] : 0.0f;
                v.z = valid ? acc[0][2] : 0.0f;
                v.w = valid ? acc[0][3] : 0.0f;
                *reinterpret_cast<float4 *>(a.yout + ((size_t)j * a.out_side + pi) * 8 + kq) = v;
            }
            continue;
        }
        const size_t base = ((size_t)j * a.out_side + pi) * COUTP;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int c0 = mb * 16 + kq;
            bf16_t h[4];
            if (EP == EP_MASK) {
                uint2 mv = make_uint2(0, 0);
                if (valid) mv = *reinterpret_cast<const uint2 *>(a.mask + ((size_t)j * a.mask_side + pi) * COUTP + c0);
                const bf16_t m[4] = {(bf16_t)(mv.x & 0xffff), (bf16_t)(mv.x >> 16), (bf16_t)(mv.y & 0xffff),
                                     (bf16_t)(mv.y >> 16)};
#pragma unroll
                for (int e = 0; e < 4; ++e) h[e] = (valid && m[e] != 0) ? bf16_rne(acc[mb][e]) : (bf16_t)0;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) h[e] = valid ? bf16_rne(fmaxf(acc[mb][e], 0.0f)) : (bf16_t)0;
            }
            *reinterpret_cast<uint2 *>(a.out + base + c0) = pack4(h[0], h[1], h[2], h[3]);
        }
    }
}

// The weight planes of a level from BoxMG's (already in C) and the network's
// outputs y (8 FP32 values per coarse point, side nc + 2): corrections that
// keep each F-point's weight sum, in FP64,
//   x-edge: e = 0.5 (y_LR - y_LL), LR += e, LL -= e;
//   y-edge: e = 0.5 (y_LA - y_LB), LA += e, LB -= e;
//   cell centre: m = 0.25 (((y_LNE + y_LNW) + y_LSE) + y_LSW), w += y_w - m;
// the weights of F-points that do not exist (x-edges in row nc + 1, y-edges in
// column nc + 1) and the row and column 0 are zero.
static __global__ void k_net_apply(Wts<double> C, int nc, const float *__restrict__ Y)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > nc + 1 || J > nc + 1) return;
    const size_t c = (size_t)J * C.ld + I;
    double *w = C.p;
    if (I == 0 || J == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) w[k * C.ps + c] = 0.0;
        return;
    }
    double y[8];
    const float *yp = Y + ((size_t)J * (nc + 2) + I) * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = (double)yp[k];
    if (J <= nc) {
        const double e = 0.5 * (y[LR] - y[LL]);
        w[LR * C.ps + c] = w[LR * C.ps + c] + e;
        w[LL * C.ps + c] = w[LL * C.ps + c] - e;
    } else {
        w[LR * C.ps + c] = 0.0;
        w[LL * C.ps + c] = 0.0;
    }
    if (I <= nc) {
        const double e = 0.5 * (y[LA] - y[LB]);
        w[LA * C.ps + c] = w[LA * C.ps + c] + e;
        w[LB * C.ps + c] = w[LB * C.ps + c] - e;
    } else {
        w[LA * C.ps + c] = 0.0;
        w[LB * C.ps + c] = 0.0;
    }
    const double m = 0.25 * (((y[LNE] + y[LNW]) + y[LSE]) + y[LSW]);
    w[LNE * C.ps + c] = w[LNE * C.ps + c] + (y[LNE] - m);
    w[LNW * C.ps + c] = w[LNW * C.ps + c] + (y[LNW] - m);
    w[LSE * C.ps + c] = w[LSE * C.ps + c] + (y[LSE] - m);
    w[LSW * C.ps + c] = w[LSW * C.ps + c] + (y[LSW] - m);
}

// dL/dy of the output layer as the layer's bfloat16 input gradient: the
// transpose of k_net_apply's map from y to the planes (the same FP64 order)
// at the valid coarse points, zeros on the ring and in channels 8..15.
static __global__ void k_net_dy(const double *__restrict__ dCi, int ldc, size_t ps, int nc, bf16_t *__restrict__ D3)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int side = nc + 3;
    if (I >= side || J >= side) return;
    bf16_t v[16] = {};
    if (I >= 1 && I <= nc + 1 && J >= 1 && J <= nc + 1) {
        double g[8], dy[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) g[k] = dCi[(size_t)k * ps + (size_t)J * ldc + I];
        const double d1 = J <= nc ? 0.5 * (g[LR] - g[LL]) : 0.0;
        dy[LR] = d1;
        dy[LL] = -d1;
        const double d2 = I <= nc ? 0.5 * (g[LA] - g[LB]) : 0.0;
        dy[LA] = d2;
        dy[LB] = -d2;
        const double m = 0.25 * (((g[LNE] + g[LNW]) + g[LSE]) + g[LSW]);
        dy[LNE] = g[LNE] - m;
        dy[LNW] = g[LNW] - m;
        dy[LSE] = g[LSE] - m;
        dy[LSW] = g[LSW] - m;
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = bf16_rne((float)dy[k]);
    }
    uint2 *dst = reinterpret_cast<uint2 *>(D3 + ((size_t)J * side + I) * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = pack4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// Weight gradient dW[t][in][out] = sum over valid output points q of
// input(centre(q) + t)[in] * delta(q)[out] and the bias gradient sum delta,
// as GEMMs over points on the matrix cores: A[out][point] = delta,
// B[point][in] = input.  Each wave sums its share of 16-point groups and
// writes one FP32 partial; k_wgrad_reduce adds the partials in a fixed order.
struct WgArgs {
    const bf16_t *in;
    int in_side;
    const bf16_t *d;
    int d_side;
    int lo, width;     // valid output points [lo, lo + width - 1]^2
    float *part;       // [wave][WG_SLOT]
};

template <int CINP, int COUTP, int STRIDE>
__global__ __launch_bounds__(256) void k_conv_wgrad(WgArgs a)
{
    constexpr int MB = COUTP / 16, NB = CINP / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gw = blockIdx.x * 4 + wave, nw = gridDim.x * 4;
    const int total = a.width * a.width;
    const int groups = (total + 15) / 16;
    const int col = lane & 15, kq = 4 * (lane >> 4);
    f32x4 acc[9][MB][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[t][mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) bsum[mb] = 0.0f;

    for (int g = gw; g < groups; g += nw) {
        int qi[4], qj[4];
        bool ok[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = g * 16 + kq + e;
            ok[e] = q < total;
            qi[e] = a.lo + (ok[e] ? q % a.width : 0);
            qj[e] = a.lo + (ok[e] ? q / a.width : 0);
        }
        bf16x4 A[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bf16_t v = ok[e] ? a.d[((size_t)qj[e] * a.d_side + qi[e]) * COUTP + mb * 16 + col] : (bf16_t)0;
                A[mb][e] = (short)v;
                bsum[mb] += bf16_f(v);
            }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dx = t % 3 - 1, dy = t / 3 - 1;
            bf16x4 B[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    bf16_t v = 0;
                    if (ok[e])
                        v = a.in[((size_t)(STRIDE * qj[e] + dy) * a.in_side + STRIDE * qi[e] + dx) * CINP + nb * 16 + col];
                    B[nb][e] = (short)v;
                }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[t][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A[mb], B[nb], acc[t][mb][nb], 0, 0, 0);
        }
    }
    float *dst = a.part + (size_t)gw * WG_SLOT;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = mb * 16 + kq + e, ci = nb * 16 + col;
                    dst[((size_t)t * COUTP + co) * CINP + ci] = acc[t][mb][nb][e];
                }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        float v = bsum[mb];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (lane < 16) dst[9 * COUTP * CINP + mb * 16 + lane] = v;
    }
}

// grad[off + (t*cin + ci)*cout + co] += sum over waves (in order) of the
// partials, in FP64; then the bias entries.
static __global__ void k_wgrad_reduce(const float *__restrict__ part, int nwaves, int cinp, int coutp, int cin,
                                      int cout, double *__restrict__ grad, int woff, int boff)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = 9 * cin * cout;
    if (g >= nw + cout) return;
    size_t src;
    int dst;
    if (g < nw) {
        const int co = g % cout, ci = (g / cout) % cin, t = g / (cout * cin);
        src = ((size_t)t * coutp + co) * cinp + ci;
        dst = woff + g;
    } else {
        const int co = g - nw;
        src = (size_t)9 * coutp * cinp + co;
        dst = boff + co;
    }
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += (double)part[(size_t)w * WG_SLOT + src];
    grad[dst] += s;
}

// ---------------------------------------------------------------------- Adam
static __global__ void k_adam(float *__restrict__ P, float *__restrict__ M, float *__restrict__ V,
                              const double *__restrict__ G, double scale, float lr, float b1, float b2,
                              float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    const float g = (float)(G[i] * scale);
    const float m = b1 * M[i] + (1.0f - b1) * g;
    const float v = b2 * V[i] + (1.0f - b2) * (g * g);
    const float mh = __fdiv_rn(m, c1);
    const float vh = __fdiv_rn(v, c2);
    P[i] = P[i] - __fdiv_rn(lr * mh, __fsqrt_rn(vh) + eps);
    M[i] = m;
    V[i] = v;
}

// ------------------------------------------------------ two-grid adjoint
// y = g / O on the interior points of colour c, 0 elsewhere.
static __global__ void k_colour_div(Lev<double> L, int c, const double *__restrict__ g, double *__restrict__ y)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const size_t p = (size_t)j * L.ld + i;
    y[p] = ((i & 1) + 2 * (j & 1) == c) ? g[p] / L.O[p] : 0.0;
}

// y = s * x on the interior.
static __global__ void k_scale(Lev<double> L, double s, const double *__restrict__ x, double *__restrict__ y)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (i > L.n || j > L.n) return;
    const size_t p = (size_t)j * L.ld + i;
    y[p] = s * x[p];
}

// dL/dCi: the weight stored at (I, J) couples fine F-point f to coarse point
// c; its derivative is alpha_f ec_c + beta_f grc_c.
static __global__ void k_grad_planes(const double *__restrict__ alpha, const double *__restrict__ beta, int ldf,
                                     const double *__restrict__ ec, const double *__restrict__ grc, Wts<double> C,
                                     int nc)
{
    const int I = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int J = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    if (I > nc + 1 || J > nc + 1) return;
    const size_t ldc = C.ld;
    const size_t fx = (size_t)(2 * J) * ldf + (2 * I - 1);       // x-edge F-point
    const size_t fy = (size_t)(2 * J - 1) * ldf + 2 * I;         // y-edge F-point
    const size_t fz = (size_t)(2 * J - 1) * ldf + (2 * I - 1);   // cell-centre F-point
    const size_t c = (size_t)J * ldc + I;
    auto d = [&](size_t f, size_t cc) { return alpha[f] * ec[cc] + beta[f] * grc[cc]; };
    C.p[LR * C.ps + c] = d(fx, c);
    C.p[LL * C.ps + c] = d(fx, c - 1);
    C.p[LA * C.ps + c] = d(fy, c);
    C.p[LB * C.ps + c] = d(fy, c - ldc);
    C.p[LNE * C.ps + c] = d(fz, c);
    C.p[LNW * C.ps + c] = d(fz, c - 1);
    C.p[LSE * C.ps + c] = d(fz, c - ldc);
    C.p[LSW * C.ps + c] = d(fz, c - ldc - 1);
}

dim3 tiles(int nx, int ny) { return grid2(nx, ny, dim3(32, 8)); }

}  // namespace

// ============================================================ network handle
struct bmg_net {
    int max_n = 0, train = 0;
    hipStream_t st = nullptr;
    float *P = nullptr, *M = nullptr, *V = nullptr;   // parameters, Adam moments
    double *G = nullptr;                              // gradient sum
    uint2 *PK = nullptr;                              // packed bfloat16 operands
    bf16_t *X = nullptr, *H1 = nullptr, *H2 = nullptr, *D3 = nullptr, *D2 = nullptr, *D1 = nullptr;
    float *Y = nullptr;                               // the output layer's FP32 values
    int *flags = nullptr;                             // breakdown bits of BoxMG's weights
    float *part = nullptr;
    double *vec = nullptr;                            // two-grid vectors
    size_t vec_cap = 0;                               // doubles in vec
    int steps = 0;
    int last_n = 0;                                   // level of the last forward pass
    bool last_nine = false;
};

namespace {

// Workspace layout of a network; with base == nullptr it only measures.
size_t net_plan(bmg_net *h, int max_n, int train, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        off = (off + ALIGN - 1) & ~(ALIGN - 1);
        char *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const size_t n = max_n, nc = (max_n - 1) / 2;
    // two-grid vectors: 12 of the fine level, then dL/dCi in the coarse weight layout
    const size_t vec_cap = 12 * (n + 2) * pitch_of((int)n) + 8 * (nc + 2) * pitch_of((int)nc);
    float *P = (float *)take(NP * 4), *M = (float *)take(NP * 4), *V = (float *)take(NP * 4);
    double *G = (double *)take(NP * 8);
    uint2 *PK = (uint2 *)take((size_t)PK_TOTAL * 8);
    bf16_t *X = (bf16_t *)take((n + 2) * (n + 2) * 16 * 2);
    bf16_t *H1 = (bf16_t *)take((n + 3) * (n + 3) * 32 * 2);
    bf16_t *H2 = (bf16_t *)take((nc + 3) * (nc + 3) * 32 * 2);
    float *Y = (float *)take((nc + 2) * (nc + 2) * 8 * 4);
    int *flags = (int *)take(64);
    bf16_t *D3 = nullptr, *D2 = nullptr, *D1 = nullptr;
    float *part = nullptr;
    double *vec = nullptr;
    if (train) {
        D3 = (bf16_t *)take((nc + 3) * (nc + 3) * 16 * 2);
        D2 = (bf16_t *)take((nc + 3) * (nc + 3) * 32 * 2);
        D1 = (bf16_t *)take((n + 2) * (n + 2) * 32 * 2);
        part = (float *)take((size_t)WG_WAVES * WG_SLOT * 4);
        vec = (double *)take(vec_cap * 8);
    }
    if (h) {
        h->P = P; h->M = M; h->V = V; h->G = G; h->PK = PK;
        h->X = X; h->H1 = H1; h->H2 = H2; h->D3 = D3; h->D2 = D2; h->D1 = D1; h->Y = Y; h->flags = flags;
        h->part = part; h->vec = vec; h->vec_cap = train ? vec_cap : 0;
    }
    return (off + ALIGN - 1) & ~(ALIGN - 1);
}

bmg_status repack(bmg_net *h)
{
    hipLaunchKernelGGL(k_pack_weights, dim3((PK_TOTAL * 4 + 255) / 256), dim3(256), 0, h->st, (const float *)h->P,
                       (bf16_t *)h->PK);
    LAUNCHCHK();
    return BMG_OK;
}

template <int CINP, int COUTP, int MODE, int EP>
bmg_status conv(bmg_net *h, ConvArgs a)
{
    const int w = a.hi - a.lo + 1;
    const int per_block = 4 * 16 * CONV_GROUPS;
    hipLaunchKernelGGL((k_conv<CINP, COUTP, MODE, EP>), dim3((w + per_block - 1) / per_block, w), dim3(256), 0, h->st,
                       a);
    LAUNCHCHK();
    return BMG_OK;
}

template <int CINP, int COUTP, int STRIDE>
bmg_status wgrad(bmg_net *h, const bf16_t *in, int in_side, const bf16_t *d, int d_side, int lo, int width,
                 int cin, int cout, int woff, int boff)
{
    const int groups = (width * width + 15) / 16;
    const int waves = std::min(WG_WAVES, std::max(4, ((groups + 3) / 4) * 4));
    WgArgs a{in, in_side, d, d_side, lo, width, h->part};
    hipLaunchKernelGGL((k_conv_wgrad<CINP, COUTP, STRIDE>), dim3(waves / 4), dim3(256), 0, h->st, a);
    const int nred = 9 * cin * cout + cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((nred + 255) / 256), dim3(256), 0, h->st, (const float *)h->part, waves,
                       CINP, COUTP, cin, cout, h->G, woff, boff);
    LAUNCHCHK();
    return BMG_OK;
}

// The weight planes of level L: BoxMG's operator-induced weights (breakdown
// bits into flags), the network, then its corrections applied.
bmg_status forward(bmg_net *h, const Lev<double> &L, bool nine, double *Ci, int ldc, size_t ps, int *flags)
{
    const int n = L.n, nc = (n - 1) / 2;
    if (n > h->max_n) return fail(BMG_EINVAL, "level of %d points exceeds the network's max_n=%d", n, h->max_n);
    const Wts<double> C{Ci, ldc, ps};
    launch_weights(L, C, nc, flags, tiles(nc + 1, nc + 1), dim3(32, 8), h->st);
    hipLaunchKernelGGL(k_net_features, tiles(n + 2, n + 2), dim3(32, 8), 0, h->st, L, nine, h->X);
    LAUNCHCHK();
    const float *P = h->P;
    ConvArgs a{};
    // conv1: fine points [1, n], written over [0, n+2] (zero ring of H1)
    a.in = h->X; a.in_side = n + 2; a.w = h->PK + PKO1; a.bias = P + OB1; a.cout = 32;
    a.lo = 0; a.hi = n + 2; a.vlo = 1; a.vhi = n; a.out = h->H1; a.out_side = n + 3;
    TRY((conv<16, 32, 0, EP_RELU>(h, a)));
    // conv2: coarse points [1, nc+1] centred on fine 2I, written over [0, nc+2]
    a = ConvArgs{};
    a.in = h->H1; a.in_side = n + 3; a.w = h->PK + PKO2; a.bias = P + OB2; a.cout = 32;
    a.lo = 0; a.hi = nc + 2; a.vlo = 1; a.vhi = nc + 1; a.out = h->H2; a.out_side = nc + 3;
    TRY((conv<32, 32, 1, EP_RELU>(h, a)));
    // conv3: the eight outputs at [1, nc+1], zeros at index 0
    a = ConvArgs{};
    a.in = h->H2; a.in_side = nc + 3; a.w = h->PK + PKO3; a.bias = P + OB3; a.cout = 8;
    a.lo = 0; a.hi = nc + 1; a.vlo = 1; a.vhi = nc + 1; a.yout = h->Y; a.out_side = nc + 2;
    TRY((conv<32, 16, 0, EP_OUT>(h, a)));
    hipLaunchKernelGGL(k_net_apply, tiles(nc + 2, nc + 2), dim3(32, 8), 0, h->st, C, nc, (const float *)h->Y);
    LAUNCHCHK();
    h->last_n = n;
    h->last_nine = nine;
    return BMG_OK;
}

bmg_status backward(bmg_net *h, const double *dCi, int ldc, size_t ps)
{
    if (!h->train) return fail(BMG_EINVAL, "the network was created for inference only");
    const int n = h->last_n, nc = (n - 1) / 2;
    if (n < 7) return fail(BMG_EINVAL, "no forward pass to differentiate");
    hipLaunchKernelGGL(k_net_dy, tiles(nc + 3, nc + 3), dim3(32, 8), 0, h->st, dCi, ldc, ps, nc, h->D3);
    LAUNCHCHK();
    // conv3: weights, then dH2 (masked by H2 > 0) -> D2
    TRY((wgrad<32, 16, 1>(h, h->H2, nc + 3, h->D3, nc + 3, 1, nc + 1, 32, 8, OW3, OB3)));
    ConvArgs a{};
    a.in = h->D3; a.in_side = nc + 3; a.w = h->PK + PKO3T; a.cout = 32;
    a.lo = 0; a.hi = nc + 2; a.vlo = 1; a.vhi = nc + 1; a.out = h->D2; a.out_side = nc + 3;
    a.mask = h->H2; a.mask_side = nc + 3;
    TRY((conv<16, 32, 2, EP_MASK>(h, a)));
    // conv2: weights, then dH1 (masked by H1 > 0) -> D1 on the fine points
    TRY((wgrad<32, 32, 2>(h, h->H1, n + 3, h->D2, nc + 3, 1, nc + 1, 32, 32, OW2, OB2)));
    a = ConvArgs{};
    a.in = h->D2; a.in_side = nc + 3; a.w = h->PK + PKO2T; a.cout = 32;
    a.lo = 1; a.hi = n; a.vlo = 1; a.vhi = n; a.out = h->D1; a.out_side = n + 2;
    a.mask = h->H1; a.mask_side = n + 3;
    TRY((conv<32, 32, 3, EP_MASK>(h, a)));
    // conv1: weights
    TRY((wgrad<16, 32, 1>(h, h->X, n + 2, h->D1, n + 2, 1, n, 9, 32, OW1, OB1)));
    return BMG_OK;
}

}  // namespace

// ================================================================== internal
namespace bmgi {

bmg_status net_level_weights(bmg_net *net, const Lev<double> &L, bool nine, const Wts<double> &C, int *flags,
                             void *stream)
{
    // run on the solver's stream, in order with the rest of its set-up
    const hipStream_t saved = net->st;
    net->st = (hipStream_t)stream;
    const bmg_status s = forward(net, L, nine, C.p, C.ld, C.ps, flags);
    net->st = saved;
    return s;
}

}  // namespace bmgi

namespace {

// Sum of squares of the padded vector x (interior of L's shape) -> scal[slot].
bmg_status vec_sumsq(bmg_solver *h, const Lev<double> &L, const double *x, int slot)
{
    const int nb = std::min(NPART_ROWS, L.n);
    hipLaunchKernelGGL((k_sumsq_partial<double, false, false>), dim3(nb), dim3(256), 0, h->st, L, x, h->part,
                       nullptr);
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(1024), 0, h->st, (const double *)h->part, nb, h->scal + slot,
                       nullptr, h->count, h->stop, (const double *)h->scal, 0.0, 0, 0.0);
    LAUNCHCHK();
    return BMG_OK;
}

void gs_sweep(bmg_solver *h, const Lev<double> &A, bool nine)
{
    for (int c = 0; c < 4; ++c) {
        const int ni = (c & 1) ? (A.n + 1) / 2 : (A.n - 1) / 2;
        const int nj = (c >> 1) ? (A.n + 1) / 2 : (A.n - 1) / 2;
        const dim3 g = grid2(ni, nj, dim3(64, 4));
        if (nine) hipLaunchKernelGGL((k_gs_colour<double, true>), g, dim3(64, 4), 0, h->st, A, c, nullptr);
        else hipLaunchKernelGGL((k_gs_colour<double, false>), g, dim3(64, 4), 0, h->st, A, c, nullptr);
    }
}

// r = b - A u with A's stencil and the given vectors.
void resid(bmg_solver *h, Lev<double> A, bool nine, const double *b, const double *u, double *r)
{
    A.b = const_cast<double *>(b);
    A.u = const_cast<double *>(u);
    A.r = r;
    const dim3 g = grid2(A.n, A.n, dim3(64, 4));
    if (nine) hipLaunchKernelGGL((k_residual<double, true>), g, dim3(64, 4), 0, h->st, A, nullptr);
    else hipLaunchKernelGGL((k_residual<double, false>), g, dim3(64, 4), 0, h->st, A, nullptr);
}

void restrict_to(bmg_solver *h, const double *r, int ldf, const Wts<double> &C, const Lev<double> &Cl)
{
    hipLaunchKernelGGL((k_restrict<double>), grid2(Cl.n, Cl.n, dim3(64, 4)), dim3(64, 4), 0, h->st, r, ldf, C, Cl,
                       nullptr);
}

void interp_into(bmg_solver *h, Lev<double> F, double *u, const Wts<double> &C, const double *ec)
{
    F.u = u;
    launch_interp_add<double>(F, C, ec, nullptr, h->st);
}

}  // namespace

namespace {
bmg_status twogrid(bmg_net *net, bmg_solver *h, const double *r0, double inner_tol, int inner_max, double *loss,
                   double *dCi);
}  // namespace

// ===================================================================== C API
extern "C" {

bmg_status bmg_net_workspace_bytes(int max_n, int train, size_t *bytes)
{
    if (!bytes) return fail(BMG_EINVAL, "bytes is NULL");
    if (!valid_n(max_n) || max_n < 7) return fail(BMG_EINVAL, "max_n=%d is not 2^m-1 >= 7", max_n);
    *bytes = net_plan(nullptr, max_n, train ? 1 : 0, nullptr);
    return BMG_OK;
}

bmg_status bmg_net_create(bmg_net **out, int max_n, int train, const float *params, void *workspace,
                          size_t ws_bytes, bmg_stream stream)
{
    if (!out) return fail(BMG_EINVAL, "out pointer is NULL");
    *out = nullptr;
    if (!params) return fail(BMG_EINVAL, "params is NULL");
    size_t need = 0;
    TRY(bmg_net_workspace_bytes(max_n, train, &need));
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace & (ALIGN - 1)))
        return fail(BMG_EWORKSPACE, "workspace %p of %zu bytes; need %zu bytes, 256-byte aligned", workspace,
                    ws_bytes, need);
    bmg_net *h = new bmg_net();
    h->max_n = max_n;
    h->train = train ? 1 : 0;
    h->st = (hipStream_t)stream;
    net_plan(h, max_n, h->train, (char *)workspace);
    auto bail = [&](bmg_status s) { delete h; return s; };
    if (hipMemsetAsync(workspace, 0, need, h->st) != hipSuccess)
        return bail(fail(BMG_EDEVICE, "clearing the network workspace failed"));
    if (hipMemcpyAsync(h->P, params, NP * sizeof(float), hipMemcpyHostToDevice, h->st) != hipSuccess)
        return bail(fail(BMG_EDEVICE, "uploading the parameters failed"));
    bmg_status s = repack(h);
    if (s != BMG_OK) return bail(s);
    if (hipStreamSynchronize(h->st) != hipSuccess) return bail(fail(BMG_EDEVICE, "network set-up failed"));
    *out = h;
    return BMG_OK;
}

bmg_status bmg_net_set_params(bmg_net *net, const float *params)
{
    if (!net || !params) return fail(BMG_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(net->P, params, NP * sizeof(float), hipMemcpyHostToDevice, net->st));
    TRY(repack(net));
    HIPCHK(hipStreamSynchronize(net->st));
    return BMG_OK;
}

bmg_status bmg_net_get_params(bmg_net *net, float *params)
{
    if (!net || !params) return fail(BMG_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(params, net->P, NP * sizeof(float), hipMemcpyDeviceToHost, net->st));
    HIPCHK(hipStreamSynchronize(net->st));
    return BMG_OK;
}

bmg_status bmg_net_destroy(bmg_net *net)
{
    delete net;
    return BMG_OK;
}

bmg_status bmg_net_forward(bmg_net *net, int n, int ld, const double *O, const double *W, const double *S,
                           const double *SW, const double *NW, double *Ci, int ldc, size_t ps)
{
    if (!net || !O || !W || !S || !Ci) return fail(BMG_EINVAL, "NULL argument");
    if (!valid_n(n) || n < 7) return fail(BMG_EINVAL, "n=%d is not 2^m-1 >= 7", n);
    if ((SW == nullptr) != (NW == nullptr)) return fail(BMG_EINVAL, "SW and NW must both be given or both NULL");
    const int nc = (n - 1) / 2;
    if (ld < n + 2 || ldc < nc + 2 || ps < (size_t)(nc + 2) * ldc) return fail(BMG_EINVAL, "bad pitch");
    Lev<double> L{};
    L.n = n;
    L.ld = ld;
    L.O = const_cast<double *>(O);
    L.W = const_cast<double *>(W);
    L.S = const_cast<double *>(S);
    L.SW = const_cast<double *>(SW);
    L.NW = const_cast<double *>(NW);
    return forward(net, L, SW != nullptr, Ci, ldc, ps, net->flags);
}

bmg_status bmg_net_backward(bmg_net *net, const double *dCi, int ldc, size_t ps)
{
    if (!net || !dCi) return fail(BMG_EINVAL, "NULL argument");
    const int nc = (net->last_n - 1) / 2;
    if (ldc < nc + 2 || ps < (size_t)(nc + 2) * ldc) return fail(BMG_EINVAL, "bad pitch");
    return backward(net, dCi, ldc, ps);
}

bmg_status bmg_net_get_grad(bmg_net *net, double *grad)
{
    if (!net || !grad) return fail(BMG_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(grad, net->G, NP * sizeof(double), hipMemcpyDeviceToHost, net->st));
    HIPCHK(hipStreamSynchronize(net->st));
    return BMG_OK;
}

bmg_status bmg_net_zero_grad(bmg_net *net)
{
    if (!net) return fail(BMG_EINVAL, "NULL argument");
    HIPCHK(hipMemsetAsync(net->G, 0, NP * sizeof(double), net->st));
    return BMG_OK;
}

bmg_status bmg_net_adam(bmg_net *net, float lr, float beta1, float beta2, float eps, double scale)
{
    if (!net) return fail(BMG_EINVAL, "NULL argument");
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(BMG_EINVAL, "bad Adam hyper-parameters");
    net->steps += 1;
    const float c1 = (float)(1.0 - pow((double)beta1, (double)net->steps));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)net->steps));
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, net->st, net->P, net->M, net->V,
                       (const double *)net->G, scale, lr, beta1, beta2, eps, c1, c2);
    LAUNCHCHK();
    return repack(net);
}

bmg_status bmg_net_export(bmg_net *net, int what, void *dst, size_t *bytes)
{
    if (!net || !bytes) return fail(BMG_EINVAL, "NULL argument");
    const size_t n = net->last_n, nc = (n - 1) / 2;
    if (n < 7) return fail(BMG_EINVAL, "no forward pass yet");
    const bf16_t *src = nullptr;
    size_t sz = 0;
    switch (what) {
    case BMG_NET_X: src = net->X; sz = (n + 2) * (n + 2) * 16; break;
    case BMG_NET_H1: src = net->H1; sz = (n + 3) * (n + 3) * 32; break;
    case BMG_NET_H2: src = net->H2; sz = (nc + 3) * (nc + 3) * 32; break;
    case BMG_NET_D3: src = net->D3; sz = (nc + 3) * (nc + 3) * 16; break;
    case BMG_NET_D2: src = net->D2; sz = (nc + 3) * (nc + 3) * 32; break;
    case BMG_NET_D1: src = net->D1; sz = (n + 2) * (n + 2) * 32; break;
    case BMG_NET_Y: src = reinterpret_cast<const bf16_t *>(net->Y); sz = (nc + 2) * (nc + 2) * 8 * 2; break;
    default: return fail(BMG_EINVAL, "unknown array %d", what);
    }
    if (!src) return fail(BMG_EINVAL, "array %d exists only in a training network", what);
    *bytes = sz * 2;
    if (dst) HIPCHK(hipMemcpyAsync(dst, src, sz * 2, hipMemcpyDeviceToDevice, net->st));
    return BMG_OK;
}

bmg_status bmg_net_twogrid(bmg_net *net, bmg_solver *h, const double *r0, double inner_tol, int inner_max,
                           double *loss, double *dCi)
{
    if (!net || !h || !r0 || !loss) return fail(BMG_EINVAL, "NULL argument");
    if (!net->train) return fail(BMG_EINVAL, "the network was created for inference only");
    if (h->opt.interp != BMG_INTERP_LEARNED || h->opt.net != net || h->opt.learned_levels != 1)
        return fail(BMG_EINVAL, "the solver was not set up with this network on level 0 only");
    if (h->opt.precision != BMG_FP64) return fail(BMG_EINVAL, "the training solver must be FP64");
    if (h->nlev < 2 || net->last_n != h->n) return fail(BMG_EINVAL, "the network's last pass is not this level's");
    if (h->n > net->max_n) return fail(BMG_EINVAL, "level larger than the network's max_n");
    if (!(inner_tol >= 0.0) || inner_max < 1) return fail(BMG_EINVAL, "bad inner solve limits");
    // the network's kernels run on the solver's stream for this sample
    const hipStream_t saved = net->st;
    net->st = h->st;
    const bmg_status s = twogrid(net, h, r0, inner_tol, inner_max, loss, dCi);
    net->st = saved;
    return s;
}

}  // extern "C"

namespace {

bmg_status twogrid(bmg_net *net, bmg_solver *h, const double *r0, double inner_tol, int inner_max, double *loss,
                   double *dCi)
{
    const Lev<double> &F = h->L[0];
    const Lev<double> &Cl = h->L[1];
    const Wts<double> &C = h->C[0];
    const bool nine = h->nine[0];
    const int n = F.n, nc = Cl.n;
    const size_t pl = (size_t)(n + 2) * F.ld;
    double *V[12];
    for (int k = 0; k < 12; ++k) V[k] = net->vec + k * pl;
    // dL/dCi in the layout of the level's weight planes (after the vectors)
    Wts<double> dC = C;
    dC.p = net->vec + 12 * pl;
    if (12 * pl + 8 * C.ps > net->vec_cap) return fail(BMG_EINVAL, "network workspace too small for this level");
    HIPCHK(hipMemsetAsync(net->vec, 0, (12 * pl + 8 * C.ps) * sizeof(double), h->st));
    hipLaunchKernelGGL((k_pack_in<double, double>), grid2(n, n, dim3(64, 4)), dim3(64, 4), 0, h->st, r0, n, V[0],
                       F.ld);
    Lev<double> A = F;
    // forward cycle: x1 = S(0), r1, rc, ec, x2 = x1 + P ec, x3 = S(x2), r3
    A.b = V[0];
    A.u = V[1];
    gs_sweep(h, A, nine);
    resid(h, F, nine, V[0], V[1], V[2]);
    restrict_to(h, V[2], F.ld, C, Cl);
    LAUNCHCHK();
    int cyc = 0;
    TRY(solve_level(h, 1, inner_tol, inner_max, &cyc));
    const size_t plc = (size_t)(nc + 2) * Cl.ld;
    HIPCHK(hipMemcpyAsync(V[10], Cl.u, plc * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    interp_into(h, F, V[1], C, V[10]);
    interp_into(h, F, V[8], C, V[10]);
    gs_sweep(h, A, nine);
    resid(h, F, nine, V[0], V[1], V[3]);
    TRY(vec_sumsq(h, F, V[0], 6));
    TRY(vec_sumsq(h, F, V[3], 7));
    double s[2];
    HIPCHK(hipMemcpyAsync(s, h->scal + 6, 2 * sizeof(double), hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    if (!(s[0] > 0.0)) return fail(BMG_EINVAL, "r0 is zero");
    *loss = s[1] / s[0];
    // adjoint: g3 = 2 r3 / ||r0||^2, gx = -A g3, the post sweep's transpose
    hipLaunchKernelGGL(k_scale, grid2(n, n, dim3(64, 4)), dim3(64, 4), 0, h->st, F, 2.0 / s[0], (const double *)V[3],
                       V[5]);
    resid(h, F, nine, V[9], V[5], V[4]);
    double *g = V[4], *gn = V[5];
    for (int c = 3; c >= 0; --c) {
        hipLaunchKernelGGL(k_colour_div, grid2(n, n, dim3(64, 4)), dim3(64, 4), 0, h->st, F, c, (const double *)g,
                           V[6]);
        resid(h, F, nine, g, V[6], gn);
        std::swap(g, gn);
    }
    restrict_to(h, g, F.ld, C, Cl);
    LAUNCHCHK();
    TRY(solve_level(h, 1, inner_tol, inner_max, &cyc));
    HIPCHK(hipMemcpyAsync(V[11], Cl.u, plc * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    interp_into(h, F, V[7], C, V[11]);
    resid(h, F, nine, g, V[7], V[6]);       // alpha = g2 - A P grc
    resid(h, F, nine, V[2], V[8], V[3]);    // beta  = r1 - A P ec
    hipLaunchKernelGGL(k_grad_planes, grid2(nc + 1, nc + 1, dim3(32, 8)), dim3(32, 8), 0, h->st,
                       (const double *)V[6], (const double *)V[3], F.ld, (const double *)V[10],
                       (const double *)V[11], dC, nc);
    LAUNCHCHK();
    if (dCi)
        HIPCHK(hipMemcpy2DAsync(dCi, (size_t)(nc + 2) * sizeof(double), dC.p, (size_t)dC.ld * sizeof(double),
                                (size_t)(nc + 2) * sizeof(double), (size_t)8 * (nc + 2), hipMemcpyDeviceToDevice,
                                h->st));
    TRY(backward(net, dC.p, dC.ld, dC.ps));
    HIPCHK(hipStreamSynchronize(h->st));
    return BMG_OK;
}

}  // namespace
