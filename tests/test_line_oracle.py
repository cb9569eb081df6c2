"""Pins of the oracle's line relaxation (the "Line" relaxation of Fig.
vcycle_flowchart, read as alternating zebra line Gauss-Seidel), checked against
what the definition and the mathematics fix: the factor reproduces each line's
matrix, one relaxation equals the block Gauss-Seidel of the explicit matrix
solved by SciPy, lines that do not couple are solved exactly, and strongly
anisotropic operators are smoothed where point relaxation fails."""
import numpy as np
import pytest

from oracle import dense, ref
from paper_2502_05279_amd import inputs


def level_ops(n=31, seed=3):
    p = inputs.jumping(n, 4, -2, 2, seed, seed + 1)
    st, rhs = ref.discretize(p.k, p.f)
    return ref.Hierarchy(st), rhs


@pytest.mark.parametrize("level", [0, 1])
def test_line_factor_is_each_lines_lu(level):
    """l and r rebuild every line's tridiagonal matrix: with m = 1/r,
    T = L U, L unit lower bidiagonal (l), U upper bidiagonal (m, c)."""
    H, _ = level_ops()
    O, W, S, SW, NW = H.op(level)
    n = H.level_n(level)
    lx, rx, ly, ry = ref.line_factor(O, W, S)
    for direction, (lf, rf) in (("x", (lx, rx)), ("y", (ly, ry))):
        for t in (1, n // 2, n):
            if direction == "x":
                pts = [(i, t) for i in range(1, n + 1)]
                nb = (1, 0)
            else:
                pts = [(t, j) for j in range(1, n + 1)]
                nb = (0, 1)
            T = np.zeros((n, n))
            for k, (i, j) in enumerate(pts):
                T[k, k] = dense.stencil_entry(O, W, S, SW, NW, i, j, 0, 0)
                if k > 0:
                    T[k, k - 1] = dense.stencil_entry(O, W, S, SW, NW, i, j, -nb[0], -nb[1])
                if k < n - 1:
                    T[k, k + 1] = dense.stencil_entry(O, W, S, SW, NW, i, j, nb[0], nb[1])
            L = np.eye(n)
            U = np.zeros((n, n))
            for k, (i, j) in enumerate(pts):
                if k > 0:
                    L[k, k - 1] = lf[j, i]
                U[k, k] = 1.0 / rf[j, i]
                if k < n - 1:
                    U[k, k + 1] = T[k, k + 1]
            assert np.abs(L @ U - T).max() <= 1e-14 * np.abs(T).max(), (direction, t)


@pytest.mark.parametrize("level", [0, 1])
def test_line_relaxation_is_the_zebra_block_gauss_seidel(level):
    """One relaxation = odd rows, even rows, odd columns, even columns, each
    set solved exactly with the others at their current values (dense matrix
    of the level, SciPy sparse solve), on a five- and a nine-point level."""
    H, _ = level_ops()
    op = H.op(level)
    n = H.level_n(level)
    f = ref.line_factor(*op[:3])
    rng = np.random.default_rng(level + 7)
    b = ref.pad(rng.standard_normal((n, n)))
    u = ref.pad(rng.standard_normal((n, n)))
    got = ref.line_relax(*op, f, b, u, 1)
    A = dense.matrix_from_compact(*op)
    want = dense.zebra_line_gs(A, dense.interior(b), dense.interior(u), n)
    assert np.abs(dense.interior(got) - want).max() <= 1e-12 * np.abs(want).max()


def anisotropic(n, ax, ay):
    """Constant-coefficient five-point operator with couplings -ax along x
    and -ay along y (Dirichlet), as a [n][n][5] stencil (S, W, O, E, N)."""
    st = np.zeros((n, n, 5))
    st[:, :, 0] = -ay
    st[:, :, 1] = -ax
    st[:, :, 2] = 2 * ax + 2 * ay
    st[:, :, 3] = -ax
    st[:, :, 4] = -ay
    st[0, :, 0] = 0.0
    st[:, 0, 1] = 0.0
    st[:, -1, 3] = 0.0
    st[-1, :, 4] = 0.0
    return st


@pytest.mark.parametrize("ax,ay", [(1.0, 0.0), (0.0, 1.0)])
def test_uncoupled_lines_are_solved_exactly(ax, ay):
    """Without couplings across lines, each half of one relaxation is a direct
    solve: the residual is at rounding level afterwards."""
    n = 31
    st = anisotropic(n, ax, ay)
    op = ref.compact_from_stencil(st)
    O, W, S, SW, NW = op
    if ax == 0.0:
        O[1:-1, 1:-1] = 2 * ay
    if ay == 0.0:
        O[1:-1, 1:-1] = 2 * ax
    f = ref.line_factor(O, W, S)
    b = ref.pad(np.random.default_rng(1).standard_normal((n, n)))
    u = ref.line_relax(O, W, S, SW, NW, f, b, np.zeros_like(b), 1)
    r = ref.residual(O, W, S, SW, NW, b, u)
    assert np.abs(r).max() <= 1e-13 * np.abs(b).max()


def test_line_relaxation_handles_strong_anisotropy():
    """x-couplings 1000 times the y-couplings: point relaxation leaves the
    V-cycle slow, line relaxation makes it fast (the reason BoxMG has it)."""
    n = 63
    st = anisotropic(n, 1000.0, 1.0)
    b = ref.pad(np.random.default_rng(2).uniform(-1, 1, (n, n)))
    rho = {}
    for sm in ("point", "line"):
        H = ref.Hierarchy(st, smoother=sm)
        u, hist = H.solve(b, tol=1e-10, max_cycles=60)
        rho[sm] = (hist[-1] / hist[0]) ** (1.0 / (len(hist) - 1))
    assert rho["line"] < 0.2 and rho["point"] > 2 * rho["line"], rho


def test_line_vcycle_converges_to_the_dense_solution():
    """Line-relaxation V-cycles on a jumping-coefficient problem reach the
    SciPy solution of the same matrix."""
    n = 31
    p = inputs.jumping(n, 4, -3, 3, 11, 12)
    st, rhs = ref.discretize(p.k, p.f)
    H = ref.Hierarchy(st, smoother="line")
    u, hist = H.solve(ref.pad(rhs), tol=1e-12, max_cycles=80)
    A = dense.matrix_from_compact(*ref.compact_from_stencil(st))
    import scipy.sparse.linalg as spla
    x = spla.spsolve(A.tocsc(), rhs.reshape(-1))
    assert hist[-1] <= 1e-12
    assert np.abs(dense.interior(u) - x).max() <= 1e-9 * np.abs(x).max()
