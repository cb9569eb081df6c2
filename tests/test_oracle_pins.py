"""Pins of the CPU oracle against closed forms, invariants, library routines
and brute force (no GPU).  Each test names what it fixes."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dense, ref
from paper_2502_05279_amd import inputs

PLANES = dict(zip(ref.WEIGHT_PLANES, range(8)))


def _op(p):
    st, rhs = ref.discretize(p.k, p.f)
    return st, rhs, ref.compact_from_stencil(st)


# ------------------------------------------------------------------ a0
def test_p1_poisson_stencil_exact():
    """k = 1: interior stencil [0,-1,0; -1,4,-1; 0,-1,0]; boundary couplings 0."""
    n = 15
    st, rhs = ref.discretize(inputs.constant_k(n), np.ones((n, n)))
    S, W, O, E, N = (st[:, :, t] for t in range(5))
    assert np.all(O == 4.0)
    assert np.all(W[:, 1:] == -1.0) and np.all(W[:, 0] == 0.0)
    assert np.all(E[:, :-1] == -1.0) and np.all(E[:, -1] == 0.0)
    assert np.all(S[1:, :] == -1.0) and np.all(S[0, :] == 0.0)
    assert np.all(N[:-1, :] == -1.0) and np.all(N[-1, :] == 0.0)
    assert np.all(rhs == 1.0 / 16**2)          # b = h^2 f, h = 1/16


def test_p1b_discretisation_is_the_edge_laplacian():
    """Random k: the stencil equals the weighted graph Laplacian assembled edge by
    edge (each edge carries the mean of its two cells)."""
    n = 15
    k = inputs.lognormal_k(n, 1.0, np.random.default_rng(3))
    st, _ = ref.discretize(k, np.zeros((n, n)))
    A = dense.matrix_from_compact(*ref.compact_from_stencil(st))
    Ae = dense.edge_laplacian(k)
    assert abs(A - Ae).max() <= 4e-16 * abs(Ae).max()
    assert abs(A - A.T).max() == 0.0


@pytest.mark.slow
def test_p11_manufactured_solution_second_order():
    """u* = sin(pi x) sin(pi y), k = 1 + sin(2 pi x) cos(2 pi y)/2 at cell centres:
    the discrete solution's max error falls like h^2."""
    errs = []
    ns = [31, 63, 127, 255]
    for n in ns:
        h = 1.0 / (n + 1)
        xc = (np.arange(n + 1) + 0.5) * h
        Xc, Yc = np.meshgrid(xc, xc)                   # [jc, ic]
        k = 1.0 + 0.5 * np.sin(2 * np.pi * Xc) * np.cos(2 * np.pi * Yc)
        x = np.arange(1, n + 1) * h
        X, Y = np.meshgrid(x, x)
        pi = np.pi
        u = np.sin(pi * X) * np.sin(pi * Y)
        kk = 1.0 + 0.5 * np.sin(2 * pi * X) * np.cos(2 * pi * Y)
        kx = pi * np.cos(2 * pi * X) * np.cos(2 * pi * Y)
        ky = -pi * np.sin(2 * pi * X) * np.sin(2 * pi * Y)
        ux = pi * np.cos(pi * X) * np.sin(pi * Y)
        uy = pi * np.sin(pi * X) * np.cos(pi * Y)
        f = -(kx * ux + ky * uy) + 2 * pi**2 * kk * u
        st, rhs = ref.discretize(k, f)
        H = ref.Hierarchy(st)
        sol, hist = H.solve(ref.pad(rhs), tol=1e-11, max_cycles=60)
        assert hist[-1] <= 1e-11
        errs.append(np.abs(sol[1:-1, 1:-1] - u).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 1.9) & (orders < 2.1)), orders


# ------------------------------------------------------------ a1 weights
def test_p2_poisson_weights_bilinear_every_level():
    """k = 1: at every level the weights toward interior coarse points are exactly
    1/2 (edge points) and 1/4 (cell centres); weights toward ring points are 0."""
    n = 63
    st, _ = ref.discretize(inputs.constant_k(n), np.zeros((n, n)))
    H = ref.Hierarchy(st)
    for l in range(H.nlev - 1):
        nc = H.level_n(l + 1)
        Ci = H.field(l, "Ci")
        LNE, LA, LNW, LR, LL, LSE, LB, LSW = Ci
        I = np.arange(nc + 2)[None, :]
        J = np.arange(nc + 2)[:, None]
        inside = lambda a, b: (a >= 1) & (a <= nc) & (b >= 1) & (b <= nc)

        def check(W, valid, ci, cj, value):
            tgt = np.where(inside(ci, cj), value, 0.0)
            assert np.all(W[valid] == np.broadcast_to(tgt, W.shape)[valid])

        xe = (I >= 1) & (I <= nc + 1) & (J >= 1) & (J <= nc)
        ye = (I >= 1) & (I <= nc) & (J >= 1) & (J <= nc + 1)
        ce = (I >= 1) & (I <= nc + 1) & (J >= 1) & (J <= nc + 1)
        xe, ye, ce = (np.broadcast_to(m, Ci[0].shape) for m in (xe, ye, ce))
        check(LL, xe, I - 1, J, 0.5)
        check(LR, xe, I, J, 0.5)
        check(LB, ye, I, J - 1, 0.5)
        check(LA, ye, I, J, 0.5)
        check(LSW, ce, I - 1, J - 1, 0.25)
        check(LSE, ce, I, J - 1, 0.25)
        check(LNW, ce, I - 1, J, 0.25)
        check(LNE, ce, I, J, 0.25)


def test_p2b_one_dimensional_coefficients_give_flux_weights():
    """k depending on x only: the x-edge weights are the 1D flux-continuity
    weights k_w/(k_w+k_e), k_e/(k_w+k_e); the y-edge weights are 1/2.  Same with
    x and y exchanged."""
    n = 31
    rng = np.random.default_rng(11)
    kcol = 10.0 ** rng.uniform(-3, 3, size=n + 1)
    for transpose in (False, True):
        k = np.tile(kcol, (n + 1, 1))
        if transpose:
            k = k.T.copy()
        st, _ = ref.discretize(k, np.zeros((n, n)))
        Ci = ref.interp_weights(*ref.compact_from_stencil(st))
        nc = (n - 1) // 2
        LL, LR, LB, LA = (Ci[PLANES[nm]] for nm in ("LL", "LR", "LB", "LA"))
        if transpose:   # exchange the roles: y-edges take the flux weights
            LL, LR, LB, LA = LB.T, LA.T, LL.T, LR.T
        for I in range(2, nc + 1):
            kw, ke = kcol[2 * I - 2], kcol[2 * I - 1]
            for J in range(1, nc + 1):
                assert LL[J, I] == pytest.approx(kw / (kw + ke), rel=4e-16, abs=0)
                assert LR[J, I] == pytest.approx(ke / (kw + ke), rel=4e-16, abs=0)
        # y-edges: 1/2 toward interior coarse points, 0 toward the ring
        assert np.allclose(LB[2:nc + 2, 1:nc + 1], 0.5, rtol=1e-15, atol=0)
        assert np.allclose(LA[1:nc + 1, 1:nc + 1], 0.5, rtol=1e-15, atol=0)
        assert np.all(LB[1, 1:nc + 1] == 0) and np.all(LA[nc + 1, 1:nc + 1] == 0)


@pytest.mark.parametrize("seed", [1, 2])
def test_p6_weight_rows_sum_to_one_inside(seed):
    """Zero-row-sum rows (two or more points from the boundary) interpolate
    constants exactly: LL+LR = LA+LB = LNE+LNW+LSE+LSW = 1 on the fine level and
    on nine-point levels; Galerkin rows sum to zero there too."""
    n = 63
    p = inputs.Problem(n, inputs.lognormal_k(n, 1.5, np.random.default_rng(seed)),
                       np.zeros((n, n)))
    st, _ = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    for l in range(H.nlev - 1):
        nc = H.level_n(l + 1)
        Ci = H.field(l, "Ci")
        sl = (slice(2, nc), slice(2, nc))
        # rounding-level deviations only: a wrong index or term is O(1) off
        assert np.abs(Ci[PLANES["LL"]][sl] + Ci[PLANES["LR"]][sl] - 1).max() < 1e-13
        assert np.abs(Ci[PLANES["LA"]][sl] + Ci[PLANES["LB"]][sl] - 1).max() < 1e-13
        corner = sum(Ci[PLANES[nm]][sl] for nm in ("LNE", "LNW", "LSE", "LSW"))
        assert np.abs(corner - 1).max() < 1e-13
        if nc >= 7:
            A = dense.matrix_from_compact(*H.op(l + 1))
            rs = np.asarray(A.sum(axis=1)).reshape(nc, nc)[2:-2, 2:-2]
            assert np.abs(rs).max() <= 1e-13 * H.op(l + 1)[0].max()


# ------------------------------------------------------------ a2 RAP
def test_p3_poisson_galerkin_closed_form():
    """k = 1: level-l Galerkin stencil = centre 8/3 + (4/3) 4^-l, edges
    -(1/3 + (2/3) 4^-l), corners -(1/3)(1 - 4^-l) at every coarse point,
    couplings to the ring zero.  All values are dyadic, so exact."""
    n = 127
    st, _ = ref.discretize(inputs.constant_k(n), np.zeros((n, n)))
    H = ref.Hierarchy(st)
    for l in range(1, H.nlev):
        q = Fraction(1, 4**l)
        centre = float(Fraction(8, 3) + Fraction(4, 3) * q)
        edge = float(-(Fraction(1, 3) + Fraction(2, 3) * q))
        corner = float(-Fraction(1, 3) * (1 - q))
        nl = H.level_n(l)
        O, W, S, SW, NW = H.op(l)
        it = slice(1, nl + 1)
        assert np.all(O[it, it] == centre)
        assert np.all(W[it, 2:nl + 1] == edge) and np.all(W[it, 1] == 0)
        assert np.all(S[2:nl + 1, it] == edge) and np.all(S[1, it] == 0)
        assert np.all(SW[2:nl + 1, 2:nl + 1] == corner)
        assert np.all(SW[1, it] == 0) and np.all(SW[it, 1] == 0)
        assert np.all(NW[1:nl, 2:nl + 1] == corner)
        assert np.all(NW[nl, it] == 0) and np.all(NW[it, 1] == 0)


@pytest.mark.parametrize("n,gen", [(7, "jump"), (15, "lognormal"), (31, "jump"), (31, "lognormal")])
def test_p5_rap_restriction_interpolation_against_matrices(n, gen):
    """The stencil RAP equals P^T A P (sparse products); restriction equals P^T r
    and interpolation P e, with P assembled row by row from the weights; on the
    five-point fine level and on nine-point levels; symmetric exactly."""
    rng = np.random.default_rng(n)
    if gen == "jump":
        p = inputs.jumping(n, 4, -2, 2, 5 + n, 6)
    else:
        p = inputs.Problem(n, inputs.lognormal_k(n, 1.5, rng), np.zeros((n, n)))
    st, _ = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    for l in range(H.nlev - 1):
        nf, nc = H.level_n(l), H.level_n(l + 1)
        op, opc, Ci = H.op(l), H.op(l + 1), H.field(l, "Ci")
        A = dense.matrix_from_compact(*op)
        P = dense.prolongation(Ci, nf)
        Ac = (P.T @ A @ P).toarray()
        Ac_st = dense.matrix_from_compact(*opc).toarray()
        scale = np.abs(op[0]).max()
        assert np.abs(Ac - Ac_st).max() <= 1e-14 * scale
        assert np.abs(Ac - Ac.T).max() <= 1e-15 * scale
        r = rng.standard_normal((nf + 2, nf + 2))
        r[0, :] = r[-1, :] = r[:, 0] = r[:, -1] = 0
        bc = ref.restrict(Ci, r)
        assert np.abs(dense.interior(bc) - P.T @ dense.interior(r)).max() <= 1e-14 * np.abs(r).max()
        e = rng.standard_normal((nc + 2, nc + 2))
        e[0, :] = e[-1, :] = e[:, 0] = e[:, -1] = 0
        u0 = rng.standard_normal((nf + 2, nf + 2))
        u0[0, :] = u0[-1, :] = u0[:, 0] = u0[:, -1] = 0
        u1 = ref.interp_add(Ci, e, u0)
        assert np.abs(dense.interior(u1 - u0) - P @ dense.interior(e)).max() <= 1e-14 * np.abs(e).max()


# --------------------------------------------------------- a3 coarse solve
def test_coarse_ldlt_matches_library_solve():
    """The square-root-free Cholesky of the coarsest 9x9 operator reproduces the
    matrix (L D L^T) and solves like numpy.linalg.solve."""
    n = 31
    p = inputs.jumping(n, 8, -3, 3, 9, 10)
    st, _ = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    L3 = H.nlev - 1
    A = dense.matrix_from_compact(*H.op(L3)).toarray()
    Lf, D = H.coarse_factor()
    assert np.allclose(np.tril(Lf), Lf) and np.all(np.diag(Lf) == 1.0) and np.all(D > 0)
    assert np.abs(Lf @ np.diag(D) @ Lf.T - A).max() <= 1e-14 * np.abs(A).max()
    b = np.random.default_rng(1).standard_normal(9)
    x = ref.ldlt_solve(Lf, D, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=0)


# ------------------------------------------------------------ a4 smoother
@pytest.mark.parametrize("level", [0, 1])
def test_p9_colour_gs_is_the_triangular_solve(level):
    """One four-colour sweep = (D + L)^-1 (b - U u) with the unknowns in colour
    order (SciPy triangular solve), on a five-point and a nine-point level."""
    n = 31
    p = inputs.jumping(n, 4, -2, 2, 3, 4)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    op = H.op(level)
    nl = H.level_n(level)
    rng = np.random.default_rng(level)
    b = ref.pad(rng.standard_normal((nl, nl)))
    u = ref.pad(rng.standard_normal((nl, nl)))
    u1 = ref.gs(*op, b, u, 1)
    A = dense.matrix_from_compact(*op)
    want = dense.colour_gs(A, dense.interior(b), dense.interior(u), nl)
    assert np.abs(dense.interior(u1) - want).max() <= 1e-13 * np.abs(want).max()


def test_gs_colour_points_have_zero_residual_after_their_update():
    """Right after a sweep the last colour (cell centres) satisfies its own
    equations: the residual there is rounding-level."""
    n = 63
    p = inputs.jumping(n, 8, -2, 2, 1, 2)
    st, rhs = ref.discretize(p.k, p.f)
    op = ref.compact_from_stencil(st)
    b = ref.pad(rhs)
    u = ref.gs(*op, b, np.zeros_like(b), 1)
    r = ref.residual(*op, b, u)
    z = r[1:-1:2, 1:-1:2]          # odd i, odd j = colour 3
    assert np.abs(z).max() <= 1e-13 * np.abs(b).max()
    assert np.abs(r[2:-1:2, 2:-1:2]).max() > 1e3 * np.abs(z).max()


# --------------------------------------------------------- a10 / a11 cycles
def test_p8_one_vcycle_is_the_dense_two_grid_map():
    """n = 7 (coarsest 3x3): one V(2,1)-cycle equals S^1 (I - P Ac^-1 P^T A) S^2
    applied to (u, b) with dense matrices."""
    n = 7
    p = inputs.jumping(n, 2, -2, 2, 21, 22)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st, 2, 1)
    rng = np.random.default_rng(5)
    u = ref.pad(rng.standard_normal((n, n)))
    b = ref.pad(rhs)
    got = H.vcycle(b, u)
    A = dense.matrix_from_compact(*H.op(0))
    P = dense.prolongation(H.field(0, "Ci"), n)
    want = dense.two_grid(A, P, dense.interior(b), dense.interior(u), n, 2, 1)
    assert np.abs(dense.interior(got) - want).max() <= 1e-14 * np.abs(want).max()


@pytest.mark.parametrize("gen,tol", [("one", 1e-12), ("mild", 1e-12), ("hard", None)])
def test_p7_vcycles_converge_to_the_dense_solution(gen, tol):
    """n = 15: cycling to stagnation reaches np.linalg.solve on the dense system."""
    n = 15
    if gen == "one":
        p = inputs.Problem(n, inputs.constant_k(n), inputs.uniform_source(n, 1))
    elif gen == "mild":
        p = inputs.jumping(n, 4, -1, 1, 31, 32)
    else:
        p = inputs.jumping(n, 4, -4, 4, 33, 34)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    u, hist = H.solve(ref.pad(rhs), tol=0.0, max_cycles=200)
    A = dense.matrix_from_compact(*H.op(0)).toarray()
    x = np.linalg.solve(A, rhs.reshape(-1))
    if tol is None:
        tol = 10 * np.linalg.cond(A) * np.finfo(float).eps
    assert np.abs(dense.interior(u) - x).max() <= tol * np.abs(x).max()


def test_p10_power_of_two_scaling_is_exact():
    """V(2^s u, 2^s b) = 2^s V(u, b) bitwise; k -> 4^s k leaves P unchanged,
    scales every coarse operator by 4^s and the cycle's iterate by 4^-s."""
    n = 63
    p = inputs.jumping(n, 8, -3, 3, 41, 42)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    b = ref.pad(rhs)
    u0 = ref.pad(np.random.default_rng(2).standard_normal((n, n)))
    v = H.vcycle(b, u0)
    assert np.array_equal(H.vcycle(8.0 * b, 8.0 * u0), 8.0 * v)
    st4, _ = ref.discretize(16.0 * p.k, p.f)
    H4 = ref.Hierarchy(st4)
    for l in range(H.nlev - 1):
        assert np.array_equal(H.field(l, "Ci"), H4.field(l, "Ci"))
    for l in range(H.nlev):
        for a, a4 in zip(H.op(l), H4.op(l)):
            if a is not None:
                assert np.array_equal(16.0 * a, a4)
    v4 = H4.vcycle(b, u0 / 16.0)
    assert np.array_equal(v4, v / 16.0)


def test_p12_poisson_127_convergence_factor():
    """Sanity (order of magnitude only): V(2,1) on the 127^2 Poisson problem
    reduces the residual by at least 5x per cycle."""
    p = inputs.poisson_127()
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    u, hist = H.solve(ref.pad(rhs), tol=0.0, max_cycles=10)
    assert len(hist) == 10
    rho = (hist[6] / hist[0]) ** (1 / 6)
    assert rho < 0.2


def test_vcycle_is_deterministic_across_thread_counts(monkeypatch):
    """The colour-parallel loops give the same bits whatever the thread count."""
    import ctypes
    n = 127
    p = inputs.jumping(n, 16, -4, 4, 51, 52)
    st, rhs = ref.discretize(p.k, p.f)
    gomp = ctypes.CDLL("libgomp.so.1")
    res = []
    for threads in (1, 4):
        gomp.omp_set_num_threads(threads)
        H = ref.Hierarchy(st)
        res.append((H.field(0, "Ci"), H.op(2)[0], H.vcycle(ref.pad(rhs), np.zeros((n + 2, n + 2)))))
    gomp.omp_set_num_threads(8)
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_lumping_only_changes_non_m_matrix_rows():
    """Moving positive off-diagonals onto the diagonal before the collapse keeps
    the weights of M-matrix rows unchanged (here all levels of a smooth field) and
    keeps the denominators positive where the Galerkin operator has positive
    off-diagonal entries (sub-cell coefficient blocks on the coarse levels)."""
    n = 255
    p = inputs.jumping(n, 16, -4, 4, 201, 202)
    st, _ = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)            # would break down without lumping
    seen_positive = False
    for l in range(H.nlev):
        O, W, S, SW, NW = H.op(l)
        for a in (W, S, SW, NW):
            if a is not None and a.max() > 0:
                seen_positive = True
    assert seen_positive
    for l in range(H.nlev - 1):
        Ci = H.field(l, "Ci")
        assert np.all(Ci >= 0) and np.all(Ci <= 1.0 + 1e-15)


# ------------------------------------------------------------ a12 refinement
def test_ir_reaches_fp64_accuracy_with_fp32_cycles():
    """FP32 V-cycles inside FP64 refinement reach a 1e-12 relative residual and
    the FP64 solution; each step contracts like the FP64 cycle would."""
    n = 127
    p = inputs.jumping(n, 16, -3, 3, 61, 62)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    b = ref.pad(rhs)
    x, hist = H.solve_ir(b, tol=1e-12, max_iter=200)
    assert hist[0] == pytest.approx(1.0) and hist[-1] <= 1e-12
    u64, h64 = H.solve(b, tol=1e-13, max_cycles=400)
    assert np.abs(x - u64).max() <= 1e-9 * np.abs(u64).max()
    assert len(hist) - 1 <= 2 * len(h64) + 5


def test_refinement_converges_below_the_fp64_floor():
    """The plain FP64 iteration stagnates at the residual floor of FP64 vectors;
    carrying the iterate as a double-FP64 pair with an accurate residual keeps
    the same contraction and goes 1e3 below it.  Before the switch the two are
    the same iteration bit for bit."""
    n = 255
    p = inputs.jumping(n, 64, -4, 4, 201, 202)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    b = ref.pad(rhs)
    u0, h0 = H.solve(b, tol=1e-17, max_cycles=60, refine_factor=0)
    floor = h0.min()
    assert floor > 1e-15                                  # plain FP64 stalls
    u1, h1 = H.solve(b, tol=1e-17, max_cycles=60, refine_factor=10**5)
    k = int(np.argmax(h1 <= 1e-12))                       # the switch cycle
    assert np.array_equal(h0[:k + 1], h1[:k + 1])
    assert h1.min() < 1e-3 * floor
    rho = (h1[k + 6] / h1[k + 1]) ** (1 / 5)              # refinement contraction
    rho0 = (h0[k] / h0[k - 5]) ** (1 / 5)                 # plain contraction
    assert abs(rho - rho0) < 0.1
    # the pair's residual is the reported one; the high part alone sits at the floor
    assert H.rel_residual(b, u1, H.xl) == pytest.approx(h1[-1], rel=1e-6)
    assert H.rel_residual(b, u1) > 10 * h1[-1]
