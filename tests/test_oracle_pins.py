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
@pytest.mark.parametrize("nc", [3, 7, 15, 31])
def test_coarse_ldlt_matches_library_solve(nc):
    """The square-root-free Cholesky of the coarsest operator (band storage,
    half-bandwidth nc + 1) reproduces the matrix (L D L^T), has no entry outside
    the band, and solves like numpy.linalg.solve."""
    n = 31
    p = inputs.jumping(n, 8, -3, 3, 9, 10)
    st, _ = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st, coarsest=nc)
    assert H.level_n(H.nlev - 1) == nc
    A = dense.matrix_from_compact(*H.op(H.nlev - 1)).toarray()
    Lb, D = H.coarse_factor()
    assert Lb.shape == (nc * nc, nc + 1) and np.all(D > 0)
    Lf = ref.band_to_dense(Lb)
    assert np.abs(Lf @ np.diag(D) @ Lf.T - A).max() <= 1e-14 * np.abs(A).max()
    # the dense factor of numpy's Cholesky has the same band: L = C diag(C)^-1
    C = np.linalg.cholesky(A)
    Lc = C / np.diag(C)
    assert np.abs(Lf - Lc).max() <= 1e-12 * np.abs(Lc).max()
    b = np.random.default_rng(1).standard_normal(nc * nc)
    x = ref.band_ldlt_solve(Lb, D, b)
    xs = np.linalg.solve(A, b)
    eps = np.finfo(float).eps
    # forward error within the condition number's bound, backward error at
    # rounding level (Cholesky is backward stable)
    assert np.linalg.norm(x - xs) <= 10 * np.linalg.cond(A) * eps * np.linalg.norm(xs)
    assert np.abs(A @ x - b).max() <= 100 * eps * np.abs(A).sum(axis=1).max() * np.abs(x).max()


def test_band_ldlt_brute_force_small():
    """On a random SPD band matrix the factor equals the textbook LDL^T (the
    same recurrences written over the dense matrix in exact rational
    arithmetic, then rounded) to a few ulps, and the solve's residual is at
    rounding level."""
    from fractions import Fraction
    rng = np.random.default_rng(7)
    m, w = 12, 3
    B = np.zeros((m, m))
    for i in range(m):
        for k in range(max(0, i - w), i):
            B[i, k] = B[k, i] = -rng.uniform(0.1, 1.0)
    A = B + np.diag(np.abs(B).sum(axis=1) + rng.uniform(0.5, 1.5, m))
    Lb, D = ref.band_ldlt_factor(ref.band_of(A, w))
    Af = [[Fraction(float(v)) for v in row] for row in A]
    L = [[Fraction(0)] * m for _ in range(m)]
    Dx = [Fraction(0)] * m
    for j in range(m):
        Dx[j] = Af[j][j] - sum(L[j][k] * L[j][k] * Dx[k] for k in range(j))
        for i in range(j + 1, m):
            L[i][j] = (Af[i][j] - sum(L[i][k] * L[j][k] * Dx[k] for k in range(j))) / Dx[j]
    Lx = np.array([[float(v) for v in row] for row in L]) + np.eye(m)
    assert np.abs(ref.band_to_dense(Lb) - Lx).max() <= 1e-14
    assert np.abs(D - np.array([float(v) for v in Dx])).max() <= 1e-14 * np.abs(D).max()
    for i in range(m):                         # nothing outside the band
        assert all(L[i][k] == 0 for k in range(0, max(0, i - w)))
    b = rng.standard_normal(m)
    x = ref.band_ldlt_solve(Lb, D, b)
    assert np.abs(A @ x - b).max() <= 1e-14 * np.abs(b).max() * np.linalg.cond(A)


def test_band_solve_updates_are_fused_and_in_column_order():
    """The band solve's recurrence, written out in exact rational arithmetic
    with one rounding to the nearest double per update (y_i - L_ij y_j as one
    fused multiply-add), then y_i / D_i, then the backward updates with k
    decreasing: equal to the oracle's solve bit for bit.  The same recurrence
    with the product rounded separately differs from it in some entry, so the
    pin tells the two roundings apart."""
    from fractions import Fraction
    rng = np.random.default_rng(11)
    m, w = 40, 7
    Lb = np.zeros((m, w))
    for i in range(m):
        for k in range(max(0, i - w), i):
            Lb[i, k - i + w] = rng.uniform(-0.9, 0.9)
    D = rng.uniform(0.5, 2.0, m)
    b = rng.standard_normal(m)

    def recurrence(fused):
        def upd(a, l, y):
            if fused:
                return float(Fraction(a) - Fraction(l) * Fraction(y))
            return float(Fraction(a) - Fraction(float(Fraction(l) * Fraction(y))))
        x = [float(v) for v in b]
        for j in range(m):
            for i in range(j + 1, min(j + w, m - 1) + 1):
                x[i] = upd(x[i], Lb[i, j - i + w], x[j])
        x = [x[i] / float(D[i]) for i in range(m)]
        for k in range(m - 1, -1, -1):
            for i in range(max(0, k - w), k):
                x[i] = upd(x[i], Lb[k, i - k + w], x[k])
        return np.array(x)

    got = ref.band_ldlt_solve(Lb, D, b)
    assert np.array_equal(got, recurrence(True))
    assert not np.array_equal(got, recurrence(False))


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


@pytest.mark.parametrize("n,nc", [(15, 7), (31, 15), (63, 31)])
def test_p8_two_grid_map_with_a_larger_direct_coarse_level(n, nc):
    """With the coarsest level one below the fine one (solved by the band
    factor), one V(2,1)-cycle is exactly the two-grid map
    S^1 (I - P Ac^-1 P^T A) S^2 with dense matrices."""
    p = inputs.jumping(n, 4, -3, 3, 23, 24)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st, 2, 1, coarsest=nc)
    assert H.nlev == 2
    rng = np.random.default_rng(n)
    u = ref.pad(rng.standard_normal((n, n)))
    b = ref.pad(rhs)
    got = H.vcycle(b, u)
    A = dense.matrix_from_compact(*H.op(0))
    P = dense.prolongation(H.field(0, "Ci"), n)
    want = dense.two_grid(A, P, dense.interior(b), dense.interior(u), n, 2, 1)
    assert np.abs(dense.interior(got) - want).max() <= 1e-12 * np.abs(want).max()


def test_single_level_hierarchy_is_the_direct_solve():
    """coarsest = n: the cycle is the direct solve itself."""
    n = 15
    p = inputs.jumping(n, 4, -2, 2, 25, 26)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st, coarsest=n)
    assert H.nlev == 1
    A = dense.matrix_from_compact(*H.op(0)).toarray()
    b = ref.pad(rhs)
    u = H.vcycle(b, np.zeros_like(b))
    xs = np.linalg.solve(A, dense.interior(b))
    assert np.abs(dense.interior(u) - xs).max() <= 1e-12 * np.abs(xs).max()


@pytest.mark.parametrize("nc", [7, 15])
def test_p7_larger_coarsest_converges_to_the_dense_solution(nc):
    """n = 31: cycling with a 7^2 or 15^2 direct coarsest level reaches the dense
    solution, and converges faster per cycle than with 3^2 on a field whose
    coefficient blocks are wider than the 3^2 level's cells resolve."""
    n = 31
    p = inputs.jumping(n, 4, -4, 4, 33, 34)
    st, rhs = ref.discretize(p.k, p.f)
    b = ref.pad(rhs)
    A = dense.matrix_from_compact(*ref.compact_from_stencil(st)).toarray()
    xs = np.linalg.solve(A, dense.interior(b))
    Hn = ref.Hierarchy(st, coarsest=nc)
    u, hist = Hn.solve(b, tol=1e-14, max_cycles=200)
    assert hist[-1] <= 1e-14
    kappa = np.linalg.cond(A)
    assert np.abs(dense.interior(u) - xs).max() <= 10 * kappa * 2.2e-16 * np.abs(xs).max()
    H3 = ref.Hierarchy(st)
    _, h3 = H3.solve(b, tol=1e-14, max_cycles=200)
    assert len(hist) <= len(h3)


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


def _worked_example_stencil(case):
    """The 7 x 7 nine-point operator of tests/golden/lump9_worked_example.txt."""
    n = 7
    st = np.zeros((n, n, 9))          # SW, S, SE, W, O, E, NW, N, NE
    offs = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
    for j in range(1, n + 1):
        for i in range(1, n + 1):
            for e, (di, dj) in enumerate(offs):
                qi, qj = i + di, j + dj
                if (di, dj) == (0, 0):
                    st[j - 1, i - 1, e] = 8.0
                elif 1 <= qi <= n and 1 <= qj <= n:
                    st[j - 1, i - 1, e] = -1.0
    # one symmetric pair of couplings set to +1: (p, entry at p, q, entry at q)
    if case == "centre":
        pairs = [((3, 3), 8, (4, 4), 0)]      # NE of (3,3) = SW of (4,4)
    else:
        pairs = [((3, 4), 6, (2, 5), 2)]      # NW of (3,4) = SE of (2,5)
    for (pi, pj), ep, (qi, qj), eq in pairs:
        st[pj - 1, pi - 1, ep] = 1.0
        st[qj - 1, qi - 1, eq] = 1.0
    return st


def test_lumping_worked_example():
    """Weights of rows with a positive coupling, computed by hand in
    tests/golden/lump9_worked_example.txt, reproduced exactly (all values are
    small rationals; the FP64 results must be their correctly rounded values)."""
    from fractions import Fraction
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "lump9_worked_example.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 8
    got = {}
    for case in ("centre", "edges"):
        O, W, S, SW, NW = ref.compact_from_stencil(_worked_example_stencil(case))
        got[case] = ref.interp_weights(O, W, S, SW, NW)
    for case, plane, I, J, num, den in rows:
        w = got[case][PLANES[plane], int(J), int(I)]
        assert w == float(Fraction(int(num), int(den))), (case, plane, I, J, w)


def test_sumsq_is_the_correctly_rounded_exact_sum():
    """The compensated sum of squares equals the exact rational sum rounded
    once (to within one unit in the last place), on data where a plain running
    sum loses every small term."""
    from fractions import Fraction
    rng = np.random.default_rng(12)
    n = 31
    r = np.zeros((n + 2, n + 2))
    vals = rng.uniform(0.5, 1.0, (n, n)) * rng.choice([-1.0, 1.0], (n, n))
    vals *= np.exp2(rng.integers(-3, 1, (n, n)))
    vals[0, 0] = 2.0 ** 27 + 1.0          # first: its square absorbs every later one
    r[1:-1, 1:-1] = vals
    exact = sum(Fraction(float(v)) ** 2 for v in vals.reshape(-1))
    got = ref.sumsq(r)
    want = float(exact)
    assert abs(Fraction(got) - exact) <= Fraction(np.spacing(want))
    plain = 0.0
    for v in vals.reshape(-1):
        plain += v * v
    assert abs(Fraction(plain) - exact) > 10 * Fraction(np.spacing(want))


def test_accurate_residual_against_exact_rationals():
    """r = b - A (x_hi + x_lo) from the error-free transformations equals the
    exact rational residual up to one rounding of the result plus a term of
    order eps^2 times the sum of |terms| (Ogita, Rump and Oishi 2005), on an
    iterate so close to the solution that the plain residual has lost most of
    its digits."""
    from fractions import Fraction
    n = 15
    p = inputs.jumping(n, 4, -3, 3, 41, 42)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st)
    op = H.op(0)
    A = dense.matrix_from_compact(*op).tocsr()
    b = ref.pad(rhs)
    xs = np.linalg.solve(A.toarray(), dense.interior(b))
    xh = ref.pad(xs.reshape(n, n))
    rng = np.random.default_rng(3)
    xl = ref.pad(xs.reshape(n, n) * rng.uniform(-1, 1, (n, n)) * 2.0 ** -60)
    H.rel_residual(b, xh, xl)
    got = dense.interior(H.field(0, "r"))
    plain = dense.interior(ref.residual(*op, b, xh))
    bi, xhi, xli = dense.interior(b), dense.interior(xh), dense.interior(xl)
    eps = 2.0 ** -53
    worst_plain = 0.0
    for row in range(n * n):
        lo, hi = A.indptr[row], A.indptr[row + 1]
        r_ex = Fraction(float(bi[row]))
        mag = Fraction(abs(float(bi[row])))
        for c, a in zip(A.indices[lo:hi], A.data[lo:hi]):
            xv = Fraction(float(xhi[c])) + Fraction(float(xli[c]))
            r_ex -= Fraction(float(a)) * xv
            mag += abs(Fraction(float(a)) * xv)
        bound = eps * abs(r_ex) + Fraction(1e-28) * mag
        assert abs(Fraction(float(got[row])) - r_ex) <= bound, row
        worst_plain = max(worst_plain, float(abs(Fraction(float(plain[row])) - r_ex) / max(abs(r_ex), 1e-300)))
    assert worst_plain > 1e-6           # the plain residual is far less accurate here


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
