// Internal declarations shared by the translation units of the library: the
// solver handle, limits, error reporting and launch helpers.
#pragma once

#include "bmg.h"
#include "bmg_fused.hpp"
#include "bmg_tile2d.hpp"
#include "bmg_line.hpp"

#include <vector>

using namespace bmg;

namespace bmgi {

constexpr int MAXL = 20;
constexpr int NPART = 8192;      // partial sums of a norm (>= fused tiles)
constexpr int NPART_ROWS = 1024; // partial sums of the row-parallel reductions
constexpr size_t ALIGN = 256;
constexpr int MAX_TRACE = 65536;

// Records a one-line description for bmg_last_error() and returns s.
bmg_status fail(bmg_status s, const char *fmt, ...);

// Interpolation weights of level L from the network (learned interpolation):
// BoxMG's weights (breakdown bits into flags) with the network's corrections.
bmg_status net_level_weights(bmg_net *net, const Lev<double> &L, bool nine, const Wts<double> &C, int *flags,
                             void *stream);

// FP64 V-cycles of the handle from level l (right-hand side L[l].b, iterate
// L[l].u from zero) until ||b - A u|| / ||b|| <= tol (accurate residual) or
// maxc cycles; *cycles receives the count.  Synchronises the stream.
bmg_status solve_level(bmg_solver *h, int l, double tol, int maxc, int *cycles);

}  // namespace bmgi

#define HIPCHK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return bmgi::fail(BMG_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

#define LAUNCHCHK()                                                                     \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess)                                                           \
            return bmgi::fail(BMG_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

namespace bmgi {

inline bool valid_n(int n) { return n >= 3 && n < (1 << 16) && ((n + 1) & n) == 0; }
inline int pitch_of(int n) { return ((n + 2) + 15) & ~15; }

inline dim3 grid2(int nx, int ny, dim3 blk) { return dim3((nx + blk.x - 1) / blk.x, (ny + blk.y - 1) / blk.y); }

}  // namespace bmgi

using bmgi::MAXL;

struct bmg_solver {
    int n = 0, kind = 5, nlev = 0;
    bmg_options opt{};
    hipStream_t st = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Lev<double> L[MAXL];
    Wts<double> C[MAXL];
    bool nine[MAXL];
    bool f32 = false;
    Lev<float> L32[MAXL];
    Wts<float> C32[MAXL];
    double *ualt[MAXL];         // second iterate buffer of each level (fused passes)
    float *ualt32[MAXL];
    int norm_parts = 0;         // partial sums left by the last fused norm
    // several right-hand sides on this hierarchy (a block solve's view; 1
    // otherwise): right-hand side k's level-l arrays start k*ks[l] elements
    // after the first's, its stop flag k*kstop ints and its norm partials
    // k*kpart doubles after
    int nrhs = 1, kstop = 0, kpart = 0;
    size_t ks[MAXL] = {};
    // line relaxation: factors of the y-lines (lfy, rfy) and, transposed, of
    // the x-lines (lfx, rfx) with the transposed W; one scratch plane
    double *lfy[MAXL] = {}, *rfy[MAXL] = {}, *lfx[MAXL] = {}, *rfx[MAXL] = {}, *WT[MAXL] = {};
    double *lineD = nullptr;
    double *B0 = nullptr;       // fine right-hand side during refinement
    double *XH = nullptr;       // double-FP64 iterate, high part
    double *XL = nullptr;       // double-FP64 iterate, low part
    double *Lb = nullptr;       // coarsest factor in band storage (m x w), D (m) right after
    double *Dd = nullptr;
    BandSolve band{};           // the factor rearranged for the one-wave solve
    double t_setup_ms = 0.0;    // host wall time of bmg_setup
    int learned_used = 0;       // levels with the network's weights (learned set-up)
    int *flags = nullptr;       // validation / breakdown bits
    double *part = nullptr;     // NPART partial sums
    double *scal = nullptr;     // scalars (see enum below)
    double *hist = nullptr;     // residual history on the device
    int *count = nullptr;       // entries in hist
    int *stop = nullptr;        // stop code of the running solve
    int hist_cap = 0;
    // graph mode: two plain cycles on the k_postpre schedule, captured once
    // and replayed while the host state (the level buffers) is the one the
    // capture started from and ended in
    hipGraphExec_t pair_exec = nullptr;
    hipStream_t cap_st = nullptr;   // the stream the capture records on (the caller's may be the null stream)
    std::vector<void *> pair_state;
    double pair_tol = -1.0, pair_refine = -1.0;
    int pair_maxc = -1;
    bool pair_off = false;      // the schedule was not periodic over two cycles
    // kernel timing
    int tr_class = -1, tr_level = -1;
    std::vector<hipEvent_t> tr_ev;
    int tr_used = 0;
    double tr_bytes = 0.0, tr_pending = 0.0;   // algorithmic bytes of the timed launches
};

namespace bmgi {
// Rows per tile of a fused pass on a level of size n: the handle's option, the
// autotuned table (bmg_tile_rows_set), else a measured default.
int tile_rows_for(const bmg_solver *h, int n, bool nine);
TileGeo tile_geo(int n, int hx, int ht);
}  // namespace bmgi


#define TRY(x)                          \
    do {                                \
        bmg_status s_ = (x);            \
        if (s_ != BMG_OK) return s_;    \
    } while (0)
