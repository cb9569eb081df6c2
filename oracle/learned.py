"""Learned interpolation: plain NumPy oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU baseline import this
module.  It shares no code with the HIP path.

The paper builds no learned component.  This oracle follows the reading the
implementation is built to, stated here once:

Network (inference).  For every fine point p of a level, the input has nine
channels: the stencil coefficients of p in the order SW, S, SE, W, O, E, NW, N,
NE, each divided by the centre coefficient O(p), rounded to FP32 and then to
bfloat16.  Three 3x3 convolutions follow:

* conv1, stride 1, 9 -> 32 channels, ReLU, at every fine interior point;
* conv2, stride 2, 32 -> 32 channels, ReLU, at the coarse points (I, J) with
  I, J = 1..nc+1, centred on the fine point (2I, 2J);
* conv3, stride 1, 32 -> 8 channels, no activation, at the same coarse points.

Each layer reads zeros outside the points the previous layer is defined on.
The eight outputs y at (I, J) are corrections to BoxMG's operator-induced
weights stored there (plane order LNE, LA, LNW, LR, LL, LSE, LB, LSW), made to
keep each F-point's weight sum, so that constants stay interpolated wherever
BoxMG interpolates them and a zero network is BoxMG itself.  In FP64, from the
FP32 outputs:

* x-edge point (LL, LR): e = 0.5 (y_LR - y_LL), LR = LR_b + e, LL = LL_b - e;
* y-edge point (LB, LA): e = 0.5 (y_LA - y_LB), LA = LA_b + e, LB = LB_b - e;
* cell centre: m = 0.25 (((y_LNE + y_LNW) + y_LSE) + y_LSW), and each of the
  four corner weights w = w_b + (y_w - m).

F-points that do not exist (the x-edge in the top row J = nc+1, the y-edge in
the right column I = nc+1) take no correction: BoxMG's zero weights stay.

Precision.  Weights and activations are bfloat16 (round to nearest, ties to
even), biases FP32.  A product of two bfloat16 numbers is exact in FP32; the
GPU adds in FP32, this oracle in FP64 (the tests bound the difference).  An
activation is bf16(fl32(relu(z))).  Gradients entering a layer's backward pass
are rounded the same way.

Training objective.  For a level operator A with interpolation P (the network's
weights) and coarse operator A_c = P^T A P (Galerkin), one two-grid cycle on
A x = r0 from x = 0: one four-colour GS sweep, residual r1, restriction
rc = P^T r1, coarse solve A_c ec = rc, x2 = x1 + P ec, one GS sweep, final
residual r3.  The loss is ||r3||^2 / ||r0||^2.  Its gradient with respect to
an interpolation weight P(i, c) (fine point i, coarse point c) is

    dL/dP(i, c) = alpha_i ec_c + beta_i grc_c,

with g2 the gradient with respect to x2 (the adjoint of the post-smoothing
sweep applied to -A (2 r3 / ||r0||^2)), grc = A_c^-1 P^T g2 (A_c is
symmetric), alpha = g2 - A P grc and beta = r1 - A P ec.  The terms come from
x2 = x1 + P ec, from rc = P^T r1 and from A_c = P^T A P respectively.

The coarse solve is by BoxMG V(2,1) cycles on the hierarchy of A_c (FP64, from
zero, until ||rc - A_c ec|| / ||rc|| <= tol) or, for the finite-difference
checks, by a dense direct solve.
"""
from __future__ import annotations

import numpy as np

from . import dense, ref

TAPS = tuple((dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1))   # t = 3(dy+1) + (dx+1)
SHAPES = (("W1", (9, 9, 32)), ("b1", (32,)), ("W2", (9, 32, 32)), ("b2", (32,)),
          ("W3", (9, 32, 8)), ("b3", (8,)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
PLANE = {"LNE": 0, "LA": 1, "LNW": 2, "LR": 3, "LL": 4, "LSE": 5, "LB": 6, "LSW": 7}


# ------------------------------------------------------------------ rounding
def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) from FP32; returns float32
    arrays holding bfloat16 values.  NaN stays NaN, overflow goes to inf."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).copy()
    out[nan] = np.nan
    return out


def act(z, rounding: bool) -> np.ndarray:
    """ReLU activation as stored: bf16(fl32(max(z, 0))) when rounding."""
    h = np.maximum(z, 0.0)
    return bf16(h).astype(np.float64) if rounding else h


def grad_in(g, rounding: bool) -> np.ndarray:
    return bf16(g).astype(np.float64) if rounding else np.asarray(g, dtype=np.float64)


# ---------------------------------------------------------------- parameters
def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name]).ravel() for name, _ in SHAPES])


def rounded(params: dict, rounding: bool) -> dict:
    """The weights as the layers use them (bfloat16), biases as FP32."""
    if not rounding:
        return params
    out = {}
    for name, v in params.items():
        out[name] = (bf16(v) if name.startswith("W") else np.float32(v)).astype(np.float64)
    return out


# ------------------------------------------------------------------ features
def stencil9(O, W, S, SW, NW) -> np.ndarray:
    """Padded compact planes -> (n, n, 9) interior stencil rows, SW..NE."""
    n = O.shape[0] - 2
    z = np.zeros_like(O)
    SWp = z if SW is None else SW
    NWp = z if NW is None else NW
    rows = [SWp[1:n + 1, 1:n + 1], S[1:n + 1, 1:n + 1], NWp[0:n, 2:n + 2],
            W[1:n + 1, 1:n + 1], O[1:n + 1, 1:n + 1], W[1:n + 1, 2:n + 2],
            NWp[1:n + 1, 1:n + 1], S[2:n + 2, 1:n + 1], SWp[2:n + 2, 2:n + 2]]
    return np.stack(rows, axis=-1)


def features(O, W, S, SW, NW, rounding: bool = True) -> np.ndarray:
    """Network input on the padded fine grid, (n+2, n+2, 9), zero ring."""
    n = O.shape[0] - 2
    a = stencil9(O, W, S, SW, NW)
    x = a / O[1:n + 1, 1:n + 1, None]
    X = np.zeros((n + 2, n + 2, 9))
    X[1:n + 1, 1:n + 1] = bf16(x).astype(np.float64) if rounding else x
    return X


# ------------------------------------------------------------------- layers
def conv(inp: np.ndarray, Wt: np.ndarray, b: np.ndarray, centres_j, centres_i) -> np.ndarray:
    """z[q] = b + sum_t inp[centre(q) + t] @ Wt[t] over the 3x3 taps, for the
    output points whose centres (in the input's padded indices) are given as
    the 1-D index arrays centres_j (rows) and centres_i (columns)."""
    cj = np.asarray(centres_j)[:, None]
    ci = np.asarray(centres_i)[None, :]
    z = np.broadcast_to(b, (cj.shape[0], ci.shape[1], b.shape[0])).astype(np.float64).copy()
    for t, (dx, dy) in enumerate(TAPS):
        z += inp[cj + dy, ci + dx] @ Wt[t]
    return z


def forward(theta: np.ndarray, O, W, S, SW=None, NW=None, rounding: bool = True) -> dict:
    """Network forward pass on one level; returns the inputs, pre-activations,
    stored activations and the eight weight planes ``Ci`` (8, nc+2, nc+2)."""
    p = rounded(unpack(theta), rounding)
    n = O.shape[0] - 2
    nc = (n - 1) // 2
    X = features(O, W, S, SW, NW, rounding)
    fine = np.arange(1, n + 1)
    z1 = conv(X, p["W1"], p["b1"], fine, fine)                    # (n, n, 32)
    H1 = np.zeros((n + 3, n + 3, 32))
    H1[1:n + 1, 1:n + 1] = act(z1, rounding)
    cen = 2 * np.arange(1, nc + 2)                                # fine centres 2I
    z2 = conv(H1, p["W2"], p["b2"], cen, cen)                     # (nc+1, nc+1, 32)
    H2 = np.zeros((nc + 3, nc + 3, 32))
    H2[1:nc + 2, 1:nc + 2] = act(z2, rounding)
    crs = np.arange(1, nc + 2)
    y = conv(H2, p["W3"], p["b3"], crs, crs)                      # (nc+1, nc+1, 8)
    if rounding:
        y = y.astype(np.float32).astype(np.float64)
    Cb = ref.interp_weights(O, W, S, SW, NW)
    Ci = corrected(Cb, y, nc)
    return {"X": X, "z1": z1, "H1": H1, "z2": z2, "H2": H2, "y": y, "Cb": Cb, "Ci": Ci,
            "n": n, "nc": nc, "params": p, "rounding": rounding}


def output_mask(nc: int) -> np.ndarray:
    """(nc+1, nc+1, 8) mask of the weights whose F-point exists."""
    m = np.ones((nc + 1, nc + 1, 8))
    m[nc, :, [PLANE["LR"], PLANE["LL"]]] = 0.0
    m[:, nc, [PLANE["LA"], PLANE["LB"]]] = 0.0
    return m


CORNERS = ("LNE", "LNW", "LSE", "LSW")


def corrected(Cb: np.ndarray, y: np.ndarray, nc: int) -> np.ndarray:
    """BoxMG's weight planes Cb plus the network's outputs y (nc+1, nc+1, 8) as
    weight-sum-preserving corrections (module docstring)."""
    Ci = Cb.copy()
    k = PLANE
    e = 0.5 * (y[..., k["LR"]] - y[..., k["LL"]])
    e[nc, :] = 0.0                                                # no x-edge point in row nc+1
    Ci[k["LR"], 1:, 1:] = Cb[k["LR"], 1:, 1:] + e
    Ci[k["LL"], 1:, 1:] = Cb[k["LL"], 1:, 1:] - e
    e = 0.5 * (y[..., k["LA"]] - y[..., k["LB"]])
    e[:, nc] = 0.0                                                # no y-edge point in column nc+1
    Ci[k["LA"], 1:, 1:] = Cb[k["LA"], 1:, 1:] + e
    Ci[k["LB"], 1:, 1:] = Cb[k["LB"], 1:, 1:] - e
    m = 0.25 * (((y[..., k["LNE"]] + y[..., k["LNW"]]) + y[..., k["LSE"]]) + y[..., k["LSW"]])
    for name in CORNERS:
        Ci[k[name], 1:, 1:] = Cb[k[name], 1:, 1:] + (y[..., k[name]] - m)
    return Ci


def correction_grad(dCi: np.ndarray, nc: int) -> np.ndarray:
    """dL/dy (nc+1, nc+1, 8) from dL/dCi: the transpose of the linear map
    y -> Ci of ``corrected`` (it is symmetric), in the same FP64 order."""
    g = np.moveaxis(dCi[:, 1:, 1:], 0, -1)
    k = PLANE
    dY = np.zeros_like(g)
    d = 0.5 * (g[..., k["LR"]] - g[..., k["LL"]])
    d[nc, :] = 0.0
    dY[..., k["LR"]], dY[..., k["LL"]] = d, -d
    d = 0.5 * (g[..., k["LA"]] - g[..., k["LB"]])
    d[:, nc] = 0.0
    dY[..., k["LA"]], dY[..., k["LB"]] = d, -d
    m = 0.25 * (((g[..., k["LNE"]] + g[..., k["LNW"]]) + g[..., k["LSE"]]) + g[..., k["LSW"]])
    for name in CORNERS:
        dY[..., k[name]] = g[..., k[name]] - m
    return dY


def bwd_conv3(fw: dict, dY: np.ndarray):
    """conv3, y(Q) = b3 + sum_t H2(Q + t) W3[t] for Q in [1, nc+1]^2: given
    dL/dy (nc+1, nc+1, 8), returns (dW3, db3, dL/dH2 on [1, nc+1]^2)."""
    p, nc, H2 = fw["params"], fw["nc"], fw["H2"]
    D3 = np.zeros((nc + 3, nc + 3, 8))
    D3[1:nc + 2, 1:nc + 2] = dY
    gW = np.stack([np.einsum("abi,abo->io", H2[1 + dy:nc + 2 + dy, 1 + dx:nc + 2 + dx], dY)
                   for dx, dy in TAPS])
    dh2 = np.zeros((nc + 1, nc + 1, 32))
    for t, (dx, dy) in enumerate(TAPS):                           # dH2(P) += W3[t] dY(P - t)
        dh2 += D3[1 - dy:nc + 2 - dy, 1 - dx:nc + 2 - dx] @ p["W3"][t].T
    return gW, dY.sum(axis=(0, 1)), dh2


def bwd_conv2(fw: dict, d2: np.ndarray):
    """conv2, z2(Q) = b2 + sum_t H1(2Q + t) W2[t]: given dL/dz2 (nc+1, nc+1,
    32), returns (dW2, db2, dL/dH1 on the fine points [1, n]^2)."""
    p, n, nc, H1 = fw["params"], fw["n"], fw["nc"], fw["H1"]
    gW = np.stack([np.einsum("abi,abo->io",
                             H1[2 + dy:2 * (nc + 1) + dy + 1:2, 2 + dx:2 * (nc + 1) + dx + 1:2], d2)
                   for dx, dy in TAPS])
    dh1 = np.zeros((n + 3, n + 3, 32))
    for t, (dx, dy) in enumerate(TAPS):                           # scatter to the fine points 2Q + t
        dh1[2 + dy:2 * (nc + 1) + dy + 1:2, 2 + dx:2 * (nc + 1) + dx + 1:2] += d2 @ p["W2"][t].T
    return gW, d2.sum(axis=(0, 1)), dh1[1:n + 1, 1:n + 1]


def bwd_conv1(fw: dict, d1: np.ndarray):
    """conv1, z1(q) = b1 + sum_t X(q + t) W1[t]: given dL/dz1 (n, n, 32),
    returns (dW1, db1)."""
    n, X = fw["n"], fw["X"]
    gW = np.stack([np.einsum("abi,abo->io", X[1 + dy:n + 1 + dy, 1 + dx:n + 1 + dx], d1)
                   for dx, dy in TAPS])
    return gW, d1.sum(axis=(0, 1))


def backward(fw: dict, dCi: np.ndarray) -> dict:
    """Gradients of a scalar with respect to the parameters, given its
    gradient ``dCi`` with respect to the weight planes: the three layers in
    reverse order, the gradient entering each rounded as specified and masked
    by the ReLU (where the stored activation is non-zero)."""
    rounding, n, nc = fw["rounding"], fw["n"], fw["nc"]
    g = {}
    dY = grad_in(correction_grad(dCi, nc), rounding)
    g["W3"], g["b3"], dh2 = bwd_conv3(fw, dY)
    live2 = (fw["H2"][1:nc + 2, 1:nc + 2] > 0) if rounding else (fw["z2"] > 0)
    d2 = grad_in(dh2 * live2, rounding)
    g["W2"], g["b2"], dh1 = bwd_conv2(fw, d2)
    live1 = (fw["H1"][1:n + 1, 1:n + 1] > 0) if rounding else (fw["z1"] > 0)
    d1 = grad_in(dh1 * live1, rounding)
    g["W1"], g["b1"] = bwd_conv1(fw, d1)
    return {"grad": pack(g), "dY": dY, "d2": d2, "d1": d1, "dh2": dh2, "dh1": dh1}


# ------------------------------------------------------------ two-grid loss
def colour_mask(n: int, c: int) -> np.ndarray:
    """Padded (n+2)^2 indicator of the interior points of colour c,
    colour(i, j) = (i mod 2) + 2 (j mod 2)."""
    j, i = np.mgrid[0:n + 2, 0:n + 2]
    m = ((i % 2) + 2 * (j % 2) == c).astype(np.float64)
    m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = 0.0
    return m


def gs_adjoint(O, W, S, SW, NW, g: np.ndarray) -> np.ndarray:
    """Transpose of the linear part of one four-colour GS sweep.  A colour-c
    step is u <- u - E_c D^-1 E_c^T A u, so its transpose is
    g <- g - A (E_c D^-1 E_c^T g); the sweep's colours 0..3 are undone 3..0."""
    n = O.shape[0] - 2
    Osafe = np.where(O != 0.0, O, 1.0)
    for c in (3, 2, 1, 0):
        y = colour_mask(n, c) * g / Osafe
        g = ref.residual(O, W, S, SW, NW, g, y)
    return g


def padded_stencil(O, W, S, SW, NW) -> np.ndarray:
    """Compact planes -> ``[n][n][9]`` stencil (the form a hierarchy is built from)."""
    return stencil9(O, W, S, SW, NW)


def coarse_solver(cO, cW, cS, cSW, cNW, tol: float, max_cycles: int, exact: bool):
    nc = cO.shape[0] - 2
    if exact:
        A = dense.matrix_from_compact(cO, cW, cS, cSW, cNW).toarray()

        def solve(rhs):
            x = np.linalg.solve(A, dense.interior(rhs))
            return dense.padded(x, nc)
        return solve, None
    H = ref.Hierarchy(padded_stencil(cO, cW, cS, cSW, cNW))

    def solve(rhs):
        if not np.any(rhs[1:-1, 1:-1]):
            return np.zeros_like(rhs)
        u, _ = H.solve(rhs, tol=tol, max_cycles=max_cycles, refine_factor=0)
        return u
    return solve, H


def grad_planes(alpha, beta, ec, grc, nc: int) -> np.ndarray:
    """dL/dCi from dL/dP(i, c) = alpha_i ec_c + beta_i grc_c, mapped to the
    storage slot of each weight (the F-point and the coarse point it feeds)."""
    d = np.zeros((8, nc + 2, nc + 2))
    J = np.arange(1, nc + 2)[:, None]
    I = np.arange(1, nc + 2)[None, :]
    # (plane, fine i, fine j, coarse I, coarse J)
    slots = (("LR", 2 * I - 1, 2 * J, I, J), ("LL", 2 * I - 1, 2 * J, I - 1, J),
             ("LA", 2 * I, 2 * J - 1, I, J), ("LB", 2 * I, 2 * J - 1, I, J - 1),
             ("LNE", 2 * I - 1, 2 * J - 1, I, J), ("LNW", 2 * I - 1, 2 * J - 1, I - 1, J),
             ("LSE", 2 * I - 1, 2 * J - 1, I, J - 1), ("LSW", 2 * I - 1, 2 * J - 1, I - 1, J - 1))
    for name, fi, fj, cI, cJ in slots:
        fi, fj, cI, cJ = np.broadcast_arrays(fi, fj, cI, cJ)
        d[PLANE[name], 1:, 1:] = alpha[fj, fi] * ec[cJ, cI] + beta[fj, fi] * grc[cJ, cI]
    return d


def twogrid(O, W, S, SW, NW, Ci, r0, tol: float = 1e-8, max_cycles: int = 30,
            exact: bool = False) -> dict:
    """Loss and dL/dCi of one two-grid cycle (arrays padded, r0 included)."""
    n = O.shape[0] - 2
    nc = (n - 1) // 2
    zero = np.zeros_like(r0)
    x1 = ref.gs(O, W, S, SW, NW, r0, zero, 1)
    r1 = ref.residual(O, W, S, SW, NW, r0, x1)
    rc = ref.restrict(Ci, r1)
    Ac = ref.rap(O, W, S, SW, NW, Ci)
    solve, H = coarse_solver(*Ac, tol=tol, max_cycles=max_cycles, exact=exact)
    ec = solve(rc)
    x2 = ref.interp_add(Ci, ec, x1)
    x3 = ref.gs(O, W, S, SW, NW, r0, x2, 1)
    r3 = ref.residual(O, W, S, SW, NW, r0, x3)
    n0 = ref.sumsq(r0)
    n3 = ref.sumsq(r3)
    loss = n3 / n0
    # adjoint
    g3 = (2.0 / n0) * r3
    gx3 = ref.residual(O, W, S, SW, NW, zero, g3)                 # -A g3
    g2 = gs_adjoint(O, W, S, SW, NW, gx3)
    gec = ref.restrict(Ci, g2)
    grc = solve(gec)
    Pg = ref.interp_add(Ci, grc, zero)
    Pe = ref.interp_add(Ci, ec, zero)
    alpha = ref.residual(O, W, S, SW, NW, g2, Pg)
    beta = ref.residual(O, W, S, SW, NW, r1, Pe)
    dCi = grad_planes(alpha, beta, ec, grc, nc)
    return {"loss": loss, "dCi": dCi, "x1": x1, "r1": r1, "rc": rc, "ec": ec, "x3": x3,
            "r3": r3, "g2": g2, "gec": gec, "grc": grc, "alpha": alpha, "beta": beta,
            "Ac": Ac, "n0": n0, "n3": n3}


def twogrid_dense_loss(O, W, S, SW, NW, Ci, r0) -> float:
    """The same loss from explicit matrices (exact coarse solve)."""
    n = O.shape[0] - 2
    A = dense.matrix_from_compact(O, W, S, SW, NW)
    P = dense.prolongation(Ci, n)
    b = dense.interior(r0)
    u = dense.two_grid(A, P, b, np.zeros_like(b), n, 1, 1)
    r = b - A.toarray() @ u
    return float(r @ r) / float(b @ b)


# -------------------------------------------------------------------- Adam
def adam(theta, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1; step counts from 1) in FP32
    arithmetic, every constant taken as its FP32 value; the bias corrections
    1 - beta^step are formed in FP64 from those values and rounded once."""
    f = np.float32
    theta, m, v, grad = (np.asarray(a, dtype=f) for a in (theta, m, v, grad))
    b1, b2, lr32, eps32 = f(beta1), f(beta2), f(lr), f(eps)
    m = b1 * m + (f(1.0) - b1) * grad
    v = b2 * v + (f(1.0) - b2) * (grad * grad)
    c1 = f(1.0 - float(b1) ** step)
    c2 = f(1.0 - float(b2) ** step)
    mh = m / c1
    vh = v / c2
    theta = theta - (lr32 * mh) / (np.sqrt(vh) + eps32)
    return theta.astype(f), m.astype(f), v.astype(f)
