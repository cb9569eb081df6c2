"""Pins of the nonsymmetric BoxMG oracle (restriction from the transposed
operator, Petrov-Galerkin coarse operators R A P, band L D U on the coarsest
level), against matrix definitions and the symmetric oracle."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import dense, ref
from paper_2502_05279_amd import inputs


def cd_stencil(n, beta, flow="rotating", block=None, lo=-1.0, hi=1.0, seed=5):
    """Convection-diffusion operator: the oracle's diffusion stencil plus the
    upwind convection part of the input generator."""
    p = inputs.jumping(n, block or max(2, (n + 1) // 8), lo, hi, seed, seed + 1)
    st, rhs = ref.discretize(p.k, p.f)
    return st + inputs.upwind_convection(n, beta, flow), rhs


def test_symmetric_operator_reduces_to_the_symmetric_oracle():
    """With A = A^T: on the fine level P and R equal the symmetric oracle's
    weights bit for bit, and so do the coarse operator's five stored
    directions while the mirrored four agree to rounding (the symmetric oracle
    copies them); below, where the coarse operators are symmetric only to
    rounding, everything agrees to rounding.  The smoother and residual are
    identical, and the solves agree to rounding with the same cycle count."""
    n = 63
    p = inputs.jumping(n, 8, -3, 3, 7, 8)
    st, rhs = ref.discretize(p.k, p.f)
    Hs, Hn = ref.Hierarchy(st), ref.NSHierarchy(st)
    assert Hs.nlev == Hn.nlev
    for l in range(Hs.nlev - 1):
        Ci, Pi, Ri = Hs.field(l, "Ci"), Hn.field(l, "Pi"), Hn.field(l, "Ri")
        if l == 0:
            assert np.array_equal(Ci, Pi) and np.array_equal(Pi, Ri)
        assert np.abs(Pi - Ci).max() <= 1e-13 and np.abs(Ri - Ci).max() <= 1e-13
        O, W, S, SW, NW = Hs.op(l + 1)
        A = Hn.planes(l + 1)
        for got, want in zip((A[4], A[3], A[1], A[0], A[6]), (O, W, S, SW, NW)):
            if l == 0:
                assert np.array_equal(got, want)
            assert np.abs(got - want).max() <= 1e-13 * np.abs(O).max()
        E = np.zeros_like(W)
        E[:, :-1] = W[:, 1:]
        N = np.zeros_like(S)
        N[:-1, :] = S[1:, :]
        assert np.abs(A[5] - E).max() <= 1e-14 * np.abs(E).max()
        assert np.abs(A[7] - N).max() <= 1e-14 * np.abs(N).max()
    planes = Hn.planes(0)
    rng = np.random.default_rng(1)
    b, u = ref.pad(rng.standard_normal((n, n))), ref.pad(rng.standard_normal((n, n)))
    assert np.array_equal(ref.ns_gs(planes, b, u, 2), ref.gs(*Hs.op(0), b, u, 2))
    assert np.array_equal(ref.ns_residual(planes, b, u), ref.residual(*Hs.op(0), b, u))
    us, hs = Hs.solve(ref.pad(rhs), tol=1e-10, max_cycles=60, refine_factor=0)
    un, hn = Hn.solve(ref.pad(rhs), tol=1e-10, max_cycles=60)
    assert len(hs) == len(hn)
    assert np.allclose(hn, hs, rtol=1e-6, atol=5e-14)   # rounding differences grow relative to a small residual
    assert np.abs(un - us).max() <= 1e-12 * np.abs(us).max()


def test_restriction_weights_are_those_of_the_transposed_operator():
    """R's weights equal the operator-induced weights of A^T formed from the
    explicitly transposed matrix, bit for bit."""
    n = 31
    st, _ = cd_stencil(n, 40.0)
    planes = ref.full_planes(st)
    A = dense.matrix_from_planes(planes)
    At = dense.planes_from_matrix(A.T.tocsr(), n)
    assert np.array_equal(ref.ns_weights(planes, transpose=True), ref.ns_weights(At))
    assert not np.array_equal(ref.ns_weights(planes, transpose=True), ref.ns_weights(planes))


@pytest.mark.parametrize("n,level", [(15, 0), (31, 0), (31, 1)])
def test_coarse_operator_is_R_A_P(n, level):
    """The coarse stencil equals the matrix product R A P (SciPy) with P from
    the interpolation weights and R the transpose of the interpolation of the
    transposed weights, on a five-point and a nine-point level."""
    st, _ = cd_stencil(n, 30.0)
    H = ref.NSHierarchy(st)
    planes = H.planes(level)
    nl = H.level_n(level)
    Pi, Ri = H.field(level, "Pi"), H.field(level, "Ri")
    A = dense.matrix_from_planes(planes)
    P = dense.prolongation(Pi, nl)
    R = dense.prolongation(Ri, nl).T
    want = (R @ A @ P).toarray()
    got = dense.matrix_from_planes(H.planes(level + 1)).toarray()
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()
    assert np.abs(got - got.T).max() > 1e-3 * np.abs(want).max()     # it is nonsymmetric


def test_band_ldu_against_textbook_and_library():
    """A random nonsymmetric band matrix: L D U rebuilds it, the factor equals
    the textbook recurrences in exact rationals (rounded) to a few ulps, the
    solve equals its recurrence in exact rationals rounded once per update bit
    for bit, and agrees with numpy.linalg.solve."""
    rng = np.random.default_rng(3)
    m, w = 30, 4
    Ad = np.zeros((m, m))
    for i in range(m):
        for k in range(max(0, i - w), min(m, i + w + 1)):
            if k != i:
                Ad[i, k] = -rng.uniform(0.0, 1.0)
    Ad += np.diag(np.abs(Ad).sum(axis=1) + rng.uniform(0.2, 1.0, m))
    Ab = np.zeros((m, 2 * w + 1))
    for i in range(m):
        for k in range(max(0, i - w), min(m, i + w + 1)):
            Ab[i, k - i + w] = Ad[i, k]
    Lb, Ub, D = ref.band_ldu_factor(Ab)
    L, U = np.eye(m), np.eye(m)
    for i in range(m):
        for k in range(max(0, i - w), i):
            L[i, k] = Lb[i, k - i + w]
        for k in range(i + 1, min(m, i + w + 1)):
            U[i, k] = Ub[i, k - i - 1]
    assert np.abs(L @ np.diag(D) @ U - Ad).max() <= 1e-14 * np.abs(Ad).max()
    # exact rationals: the same recurrences, then rounded
    a = [[Fraction(float(v)) for v in row] for row in Ad]
    for k in range(m):
        for i in range(k + 1, m):
            lik = a[i][k] / a[k][k]
            for j in range(k + 1, m):
                a[i][j] = a[i][j] - lik * a[k][j]
    Dx = np.array([float(a[k][k]) for k in range(m)])
    assert np.abs(D - Dx).max() <= 1e-14 * np.abs(D).max()
    b = rng.standard_normal(m)
    x = ref.band_ldu_solve(Lb, Ub, D, b)
    y = [float(v) for v in b]
    for j in range(m):
        for i in range(j + 1, min(j + w, m - 1) + 1):
            y[i] = float(Fraction(y[i]) - Fraction(Lb[i, j - i + w]) * Fraction(y[j]))
    y = [y[i] / float(D[i]) for i in range(m)]
    for k in range(m - 1, -1, -1):
        for i in range(max(0, k - w), k):
            y[i] = float(Fraction(y[i]) - Fraction(Ub[i, k - i - 1]) * Fraction(y[k]))
    assert np.array_equal(x, np.array(y))
    ref_x = np.linalg.solve(Ad, b)
    assert np.abs(x - ref_x).max() <= 1e-13 * np.abs(ref_x).max() * np.linalg.cond(Ad)


def test_gs_is_the_colour_ordered_triangular_solve():
    n = 31
    st, _ = cd_stencil(n, 60.0)
    H = ref.NSHierarchy(st)
    for level in (0, 1):
        planes = H.planes(level)
        nl = H.level_n(level)
        rng = np.random.default_rng(level)
        b, u = ref.pad(rng.standard_normal((nl, nl))), ref.pad(rng.standard_normal((nl, nl)))
        got = dense.interior(ref.ns_gs(planes, b, u, 1))
        want = dense.colour_gs(dense.matrix_from_planes(planes), dense.interior(b), dense.interior(u), nl)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("n", [15, 31])
def test_vcycle_with_a_direct_coarse_level_is_the_two_grid_map(n):
    """Coarsest level one below the fine one: one cycle is the explicit
    Petrov-Galerkin two-grid map (exact coarse solve)."""
    st, rhs = cd_stencil(n, 25.0)
    H = ref.NSHierarchy(st, coarsest=(n - 1) // 2)
    assert H.nlev == 2
    planes = H.planes(0)
    A = dense.matrix_from_planes(planes)
    P = dense.prolongation(H.field(0, "Pi"), n)
    R = dense.prolongation(H.field(0, "Ri"), n).T
    rng = np.random.default_rng(n)
    u0 = ref.pad(rng.standard_normal((n, n)))
    b = ref.pad(rhs)
    u1, _ = H.solve(b, u0, tol=0.0, max_cycles=1)
    want = dense.two_grid_pg(A, P, R, dense.interior(b), dense.interior(u0), n, 2, 1)
    assert np.abs(dense.interior(u1) - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("beta,flow", [(10.0, "rotating"), (80.0, "rotating"), (80.0, "constant")])
def test_convection_diffusion_converges_to_the_direct_solution(beta, flow):
    """V(2,1) cycles on convection-diffusion operators (cell Peclet number up
    to about 1) converge at a factor below 0.3 per cycle to the direct
    solution of the nonsymmetric system."""
    n = 127
    st, rhs = cd_stencil(n, beta, flow, block=16)
    H = ref.NSHierarchy(st)
    u, hist = H.solve(ref.pad(rhs), tol=1e-11, max_cycles=60)
    assert hist[-1] <= 1e-11
    rho = (hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1))
    assert rho < 0.3, rho
    A = dense.matrix_from_planes(ref.full_planes(st))
    import scipy.sparse.linalg as spla
    x = spla.spsolve(A.tocsc(), rhs.reshape(-1))
    assert np.abs(dense.interior(u) - x).max() <= 1e-8 * np.abs(x).max()
