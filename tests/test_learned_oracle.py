"""Pins of the learned-interpolation oracle (CPU only).

Each test checks the oracle against something other than itself: a library
rounding routine, brute-force loops, a symmetry the network must have, finite
differences, the explicit-matrix two-grid map, or a closed form.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import dense, learned, ref
from paper_2502_05279_amd import inputs


def _level(n: int, seed: int, nine: bool):
    """Padded planes of a 5-point fine operator, or of its Galerkin level 1."""
    p = inputs.jumping(n if not nine else 2 * n + 1, 2, -2.0, 2.0, seed, seed + 1)
    st, _ = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    return H.op(1 if nine else 0)


# ------------------------------------------------------------------ bf16
def test_bf16_rounding_special_values():
    one = 1.0
    ulp = 2.0 ** -7
    cases = {
        one: one,
        one + 2.0 ** -8: one,                          # tie -> even (down)
        one + ulp + 2.0 ** -8: one + 2 * ulp,          # tie -> even (up)
        one + 2.0 ** -8 + 2.0 ** -20: one + ulp,       # above the tie
        -(one + 2.0 ** -8 + 2.0 ** -20): -(one + ulp),
        3.4e38: np.inf,                                # past the largest bf16 + half an ulp
        3.0e38: 3.0040553e38,                          # below it: finite
        0.0: 0.0,
    }
    got = learned.bf16(np.array(list(cases), dtype=np.float64))
    assert np.array_equal(got, np.array(list(cases.values()), dtype=np.float32))
    assert np.isnan(learned.bf16(np.array([np.nan]))[0])


def test_bf16_matches_library_conversion():
    rng = np.random.default_rng(5)
    bits = rng.integers(0, 2 ** 32, size=200_000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    ours = learned.bf16(x)
    lib = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours, lib)


# ------------------------------------------------------------- features
def test_features_constant_poisson():
    n = 7
    st, _ = ref.discretize(np.ones((n + 1, n + 1)), np.zeros((n, n)))
    O, W, S, SW, NW = ref.compact_from_stencil(st)
    X = learned.features(O, W, S, SW, NW)
    mid = X[4, 4]                                  # interior point away from the ring
    assert np.array_equal(mid, np.array([0, -0.25, 0, -0.25, 1, -0.25, 0, -0.25, 0], dtype=float))
    corner = X[1, 1]                               # couplings to the boundary are zero
    assert np.array_equal(corner, np.array([0, 0, 0, 0, 1, -0.25, 0, -0.25, 0], dtype=float))
    assert not X[0].any() and not X[:, 0].any() and not X[-1].any()


# ------------------------------------------------------------ forward
def _brute_forward(theta, O, W, S, SW, NW):
    """The network written out point by point, tap by tap and channel by
    channel with Python loops (bfloat16 rounding as specified)."""
    p = learned.rounded(learned.unpack(theta), True)
    n = O.shape[0] - 2
    nc = (n - 1) // 2
    X = learned.features(O, W, S, SW, NW)

    H1 = {}
    for j in range(1, n + 1):
        for i in range(1, n + 1):
            out = []
            for o in range(32):
                s = p["b1"][o]
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        t = 3 * (dy + 1) + (dx + 1)
                        for c in range(9):
                            s += X[j + dy, i + dx, c] * p["W1"][t, c, o]
                out.append(s)
            H1[j, i] = learned.act(np.array(out), True)
    H2 = {}
    for J in range(1, nc + 2):
        for I in range(1, nc + 2):
            out = np.array(p["b2"], dtype=float)
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    t = 3 * (dy + 1) + (dx + 1)
                    v = H1.get((2 * J + dy, 2 * I + dx))
                    if v is not None:
                        for c in range(32):
                            out = out + v[c] * p["W2"][t, c]
            H2[J, I] = learned.act(out, True)
    # BoxMG's weights, then each F-point's corrections written out: the x-edge
    # pair (LL 4, LR 3), the y-edge pair (LB 6, LA 1), the corners (0, 2, 5, 7)
    Cb = ref.interp_weights(O, W, S, SW, NW)
    Ci = Cb.copy()
    for J in range(1, nc + 2):
        for I in range(1, nc + 2):
            out = np.array(p["b3"], dtype=float)
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    t = 3 * (dy + 1) + (dx + 1)
                    v = H2.get((J + dy, I + dx))
                    if v is not None:
                        for c in range(32):
                            out = out + v[c] * p["W3"][t, c]
            y = [float(np.float32(v)) for v in out]
            if J <= nc:                            # the x-edge point (2I-1, 2J) exists
                e = 0.5 * (y[3] - y[4])
                Ci[3, J, I] = Cb[3, J, I] + e
                Ci[4, J, I] = Cb[4, J, I] - e
            if I <= nc:                            # the y-edge point (2I, 2J-1) exists
                e = 0.5 * (y[1] - y[6])
                Ci[1, J, I] = Cb[1, J, I] + e
                Ci[6, J, I] = Cb[6, J, I] - e
            m = 0.25 * (((y[0] + y[2]) + y[5]) + y[7])
            for k in (0, 2, 5, 7):
                Ci[k, J, I] = Cb[k, J, I] + (y[k] - m)
    return Ci


@pytest.mark.parametrize("nine", [False, True])
def test_forward_matches_brute_force(nine):
    planes = _level(7, 11, nine)
    theta = inputs.net_random(3)
    fw = learned.forward(theta, *planes)
    ref_ci = _brute_forward(theta, *planes)
    assert np.allclose(fw["Ci"], ref_ci, rtol=1e-6, atol=1e-6)


def test_forward_translation_equivariance():
    """Shifting the fine operator by two points shifts the weights by one
    coarse point (away from the boundary the network only sees the stencils)."""
    n = 31
    rng = np.random.default_rng(9)
    k = 10.0 ** rng.uniform(-1, 1, size=(n + 3, n + 3))
    stA, _ = ref.discretize(k[:n + 1, :n + 1], np.zeros((n, n)))
    stB, _ = ref.discretize(k[2:, 2:], np.zeros((n, n)))
    theta = inputs.net_random(4)
    A = learned.forward(theta, *ref.compact_from_stencil(stA))["Ci"]
    B = learned.forward(theta, *ref.compact_from_stencil(stB))["Ci"]
    # coarse point (I, J) of B sees the stencils of coarse (I+1, J+1) of A;
    # compare where both receptive fields (+-4 fine points) are inside the grid
    assert np.array_equal(B[:, 3:12, 3:12], A[:, 4:13, 4:13])


@pytest.mark.parametrize("nine", [False, True])
def test_zero_network_gives_boxmg_weights(nine):
    """The outputs are corrections: a zero network leaves BoxMG's
    operator-induced weights exactly (the start of training)."""
    planes = _level(15, 2, nine)
    Ci = learned.forward(np.zeros(learned.NPARAM, np.float32), *planes)["Ci"]
    assert np.array_equal(Ci, ref.interp_weights(*planes))
    Ci = learned.forward(inputs.net_init(5), *planes)["Ci"]
    assert np.array_equal(Ci, ref.interp_weights(*planes))


@pytest.mark.parametrize("nine", [False, True])
def test_corrections_keep_each_points_weight_sum(nine):
    """Whatever the network outputs, each F-point's weights sum to BoxMG's sum
    (up to the rounding of the additions), so a constant is interpolated
    wherever BoxMG interpolates it; the weights of missing F-points and of
    the ring stay zero."""
    planes = _level(31, 7, nine)
    fw = learned.forward(inputs.net_random(8), *planes)
    Ci, Cb, nc = fw["Ci"], fw["Cb"], fw["nc"]
    assert np.abs(Ci - Cb).max() > 1e-3                   # the network does change them
    k = learned.PLANE
    for pair in (("LR", "LL"), ("LA", "LB"), ("LNE", "LNW", "LSE", "LSW")):
        got = sum(Ci[k[q]] for q in pair)
        want = sum(Cb[k[q]] for q in pair)
        assert np.abs(got - want).max() <= 4e-16 * (1 + np.abs(Ci[[k[q] for q in pair]]).sum(axis=0)).max()
    assert not Ci[[k["LR"], k["LL"]], nc + 1, :].any() and not Ci[[k["LA"], k["LB"]], :, nc + 1].any()
    assert not Ci[:, 0, :].any() and not Ci[:, :, 0].any()


# ----------------------------------------------------------- backward
@pytest.mark.parametrize("nine", [False, True])
def test_backward_matches_finite_differences(nine):
    """FP64 without rounding: sum(G * Ci(theta)) differentiated both ways."""
    planes = _level(7, 21, nine)
    theta = inputs.net_random(6).astype(np.float64)
    rng = np.random.default_rng(7)
    fw = learned.forward(theta, *planes, rounding=False)
    G = rng.standard_normal(fw["Ci"].shape)
    grad = learned.backward(fw, G)["grad"]
    idx = rng.choice(learned.NPARAM, size=60, replace=False)
    idx = np.concatenate([idx, [0, 2591, 2592 + 3, learned.NPARAM - 1, learned.NPARAM - 9]])
    h = 1e-6
    for t in idx:
        tp = theta.copy()
        tp[t] += h
        tm = theta.copy()
        tm[t] -= h
        fp = np.sum(G * learned.forward(tp, *planes, rounding=False)["Ci"])
        fm = np.sum(G * learned.forward(tm, *planes, rounding=False)["Ci"])
        fd = (fp - fm) / (2 * h)
        assert abs(fd - grad[t]) <= 1e-6 * max(1.0, abs(fd)), (t, fd, grad[t])


def test_backward_weight_gradient_brute_force():
    """dW3 and db3 with rounding on, summed by explicit loops."""
    planes = _level(7, 31, True)
    theta = inputs.net_random(8)
    fw = learned.forward(theta, *planes)
    G = np.random.default_rng(1).standard_normal(fw["Ci"].shape)
    bw = learned.backward(fw, G)
    g = learned.unpack(bw["grad"])
    nc = fw["nc"]
    dY = bw["dY"]
    W3 = np.zeros((9, 32, 8))
    for J in range(nc + 1):
        for I in range(nc + 1):
            for t, (dx, dy) in enumerate(learned.TAPS):
                W3[t] += np.outer(fw["H2"][J + 1 + dy, I + 1 + dx], dY[J, I])
    assert np.allclose(g["W3"], W3, rtol=1e-12, atol=1e-14)
    assert np.allclose(g["b3"], dY.sum(axis=(0, 1)), rtol=1e-12, atol=1e-14)
    # masked weights carry no gradient
    assert not dY[nc, :, [3, 4]].any() and not dY[:, nc, [1, 6]].any()


# -------------------------------------------------------- two-grid loss
def test_gs_adjoint_is_the_transpose():
    n = 15
    O, W, S, SW, NW = _level(n, 41, True)
    rng = np.random.default_rng(2)
    x = ref.pad(rng.standard_normal((n, n)))
    y = ref.pad(rng.standard_normal((n, n)))
    zero = np.zeros_like(x)
    Mx = ref.gs(O, W, S, SW, NW, zero, x, 1)                      # linear part of a sweep
    MTy = learned.gs_adjoint(O, W, S, SW, NW, y)
    lhs = np.sum(Mx * y)
    rhs = np.sum(x * MTy)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(Mx * y))
    A = dense.matrix_from_compact(O, W, S, SW, NW)
    M, _ = dense.gs_matrix(A, n)
    assert np.allclose(dense.interior(MTy), M.T @ dense.interior(y), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("nine", [False, True])
def test_twogrid_loss_matches_dense_two_grid(nine):
    n = 15
    O, W, S, SW, NW = _level(n, 51, nine)
    Ci = ref.interp_weights(O, W, S, SW, NW)
    r0 = ref.pad(inputs.residual_probe(n, 3))
    got = learned.twogrid(O, W, S, SW, NW, Ci, r0, exact=True)["loss"]
    want = learned.twogrid_dense_loss(O, W, S, SW, NW, Ci, r0)
    assert abs(got - want) <= 1e-12 * want
    assert got < 1.0
    it = learned.twogrid(O, W, S, SW, NW, Ci, r0, tol=1e-13, max_cycles=60)["loss"]
    assert abs(it - want) <= 1e-9 * want


@pytest.mark.parametrize("nine", [False, True])
def test_twogrid_gradient_matches_finite_differences(nine):
    n = 15
    O, W, S, SW, NW = _level(n, 61, nine)
    rng = np.random.default_rng(4)
    Ci = ref.interp_weights(O, W, S, SW, NW)
    nc = Ci.shape[1] - 2
    live = np.zeros_like(Ci)
    live[:, 1:, 1:] = np.moveaxis(learned.output_mask(nc), -1, 0)
    Ci = Ci + 0.05 * rng.standard_normal(Ci.shape) * live
    r0 = ref.pad(inputs.residual_probe(n, 5))
    d = learned.twogrid(O, W, S, SW, NW, Ci, r0, exact=True)["dCi"]
    h = 1e-6
    picks = [(k, J, I) for k in range(8) for J in range(1, nc + 2) for I in range(1, nc + 2)
             if live[k, J, I]]
    picks = [picks[t] for t in rng.choice(len(picks), size=40, replace=False)]
    for k, J, I in picks:
        cp = Ci.copy()
        cp[k, J, I] += h
        cm = Ci.copy()
        cm[k, J, I] -= h
        fd = (learned.twogrid_dense_loss(O, W, S, SW, NW, cp, r0)
              - learned.twogrid_dense_loss(O, W, S, SW, NW, cm, r0)) / (2 * h)
        assert abs(fd - d[k, J, I]) <= 1e-6 * max(abs(fd), 1e-3), (k, J, I, fd, d[k, J, I])
    # weights of F-points that do not exist, or feed the boundary, get nothing
    assert not d[[3, 4], nc + 1, :].any() and not d[[1, 6], :, nc + 1].any()
    assert not d[4, :, 1].any() and not d[6, 1, :].any()


def test_end_to_end_gradient_matches_finite_differences():
    """Network + two-grid loss in FP64 without rounding, exact coarse solve."""
    n = 15
    O, W, S, SW, NW = _level(n, 71, False)
    r0 = ref.pad(inputs.residual_probe(n, 6))
    theta = (inputs.net_random(12) * 0.5).astype(np.float64)

    def loss(th):
        fw = learned.forward(th, O, W, S, SW, NW, rounding=False)
        return learned.twogrid(O, W, S, SW, NW, fw["Ci"], r0, exact=True), fw

    tg, fw = loss(theta)
    grad = learned.backward(fw, tg["dCi"])["grad"]
    rng = np.random.default_rng(8)
    h = 1e-6
    for t in rng.choice(learned.NPARAM, size=25, replace=False):
        tp = theta.copy()
        tp[t] += h
        tm = theta.copy()
        tm[t] -= h
        fd = (loss(tp)[0]["loss"] - loss(tm)[0]["loss"]) / (2 * h)
        assert abs(fd - grad[t]) <= 2e-6 * max(abs(fd), 1e-4), (t, fd, grad[t])


def test_boxmg_weights_beat_zero_weights():
    """Injection-only interpolation (a zero network) reduces the residual far
    less than the operator-induced weights on a jumping-coefficient level."""
    n = 31
    O, W, S, SW, NW = _level(n, 81, False)
    r0 = ref.pad(inputs.residual_probe(n, 7))
    Ci = ref.interp_weights(O, W, S, SW, NW)
    good = learned.twogrid(O, W, S, SW, NW, Ci, r0, tol=1e-10)["loss"]
    zero = learned.twogrid(O, W, S, SW, NW, np.zeros_like(Ci), r0, tol=1e-10)["loss"]
    assert good < 0.25 * zero


# ------------------------------------------------------------------ Adam
def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    theta = rng.standard_normal(1000).astype(np.float32)
    g = rng.standard_normal(1000).astype(np.float32)
    z = np.zeros_like(theta)
    t1, m1, v1 = learned.adam(theta, z, z, g, 1, lr=1e-3)
    # after one step m_hat = g and v_hat = g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(t1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=2e-7)
    # the constants enter as FP32 values: 1 - fl32(0.999) = 1.0000467e-3
    b2 = float(np.float32(0.999))
    assert np.allclose(m1, 0.1 * g, rtol=1e-6) and np.allclose(v1, (1.0 - b2) * g * g, rtol=1e-6)
    # a zero gradient leaves everything unchanged
    t2, m2, v2 = learned.adam(theta, z, z, z, 1, lr=1e-3)
    assert np.array_equal(t2, theta) and not m2.any() and not v2.any()


def test_adam_several_steps_follow_the_real_arithmetic_update():
    """Five Adam steps (Kingma and Ba, Algorithm 1) in the oracle's FP32 against
    the same recurrence in FP64 on the FP32 values of the constants: equal to
    the accumulated FP32 rounding (a few ulps of each quantity)."""
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(2000).astype(np.float32)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
    lr, eps = float(np.float32(1e-3)), float(np.float32(1e-8))
    th64, m64, v64 = theta.astype(np.float64), np.zeros(2000), np.zeros(2000)
    for t in range(1, 6):
        g = rng.standard_normal(2000).astype(np.float32)
        theta, m, v = learned.adam(theta, m, v, g, t, lr=1e-3)
        g64 = g.astype(np.float64)
        m64 = b1 * m64 + (1 - b1) * g64
        v64 = b2 * v64 + (1 - b2) * g64 * g64
        mh, vh = m64 / (1 - b1 ** t), v64 / (1 - b2 ** t)
        th64 = th64 - lr * mh / (np.sqrt(vh) + eps)
        assert np.allclose(m, m64, rtol=1e-5, atol=1e-7)
        assert np.allclose(v, v64, rtol=1e-5, atol=1e-9)
        assert np.abs(theta - th64).max() <= 1e-6

