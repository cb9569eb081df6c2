"""Matrix tier of the CPU oracle (test infrastructure only; small grids).

Restates the objects of the method as explicit sparse or dense matrices, built
from their definitions rather than from the stencil loops of the C tier, so
that the C tier can be checked against them:

* ``edge_laplacian``: the discrete operator of -div(k grad u) (Section 2, Eq. 1)
  assembled edge by edge as a weighted graph Laplacian: each grid edge carries
  the mean of the two cells that share it, Dirichlet neighbours drop out;
* ``matrix_from_compact``: the global matrix a compact stencil stands for
  (the per-point nine-point stencil of Fig. stencil_operator);
* ``prolongation``: the interpolation operator P as a matrix, row by row from
  the F-point formulas (coarse points inject, edges take two coarse
  neighbours, cell centres four);
* ``colour_gs``: one four-colour Gauss-Seidel sweep as the triangular solve
  (D + L) u_new = b - U u_old in colour order, done by SciPy;
* ``two_grid``: the explicit two-grid map S^nu2 (I - P A_c^-1 P^T A) S^nu1;
* ``zebra_line_gs``: one alternating zebra line relaxation as four block
  Gauss-Seidel steps over the unknown sets odd rows, even rows, odd columns,
  even columns, each solved exactly (A restricted to a set is block diagonal
  with one tridiagonal block per line) by SciPy.

Unknowns are numbered k = (i-1) + n (j-1) over the interior.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _idx(n, i, j):
    return (i - 1) + n * (j - 1)


def edge_laplacian(k: np.ndarray) -> sp.csr_matrix:
    """Vertex-centred finite-volume matrix from cell coefficients ``k[jc, ic]``."""
    n = k.shape[0] - 1
    rows, cols, vals = [], [], []
    diag = np.zeros(n * n)

    def edge(p, q, kappa):
        # p interior; q interior or on the boundary ring
        (pi, pj), (qi, qj) = p, q
        a = _idx(n, pi, pj)
        diag[a] += kappa
        if 1 <= qi <= n and 1 <= qj <= n:
            rows.append(a)
            cols.append(_idx(n, qi, qj))
            vals.append(-kappa)

    for j in range(1, n + 1):
        for i in range(1, n + 1):
            # horizontal edge to (i+1, j): cells (i, j-1) and (i, j)
            edge((i, j), (i + 1, j), 0.5 * (k[j - 1, i] + k[j, i]))
            edge((i, j), (i - 1, j), 0.5 * (k[j - 1, i - 1] + k[j, i - 1]))
            edge((i, j), (i, j + 1), 0.5 * (k[j, i - 1] + k[j, i]))
            edge((i, j), (i, j - 1), 0.5 * (k[j - 1, i - 1] + k[j - 1, i]))
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n * n, n * n)).tocsr()
    return (A + sp.diags(diag)).tocsr()


_DIRS = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]


def stencil_entry(O, W, S, SW, NW, i, j, di, dj):
    """Signed matrix entry of the compact stencil at (i,j) toward (i+di, j+dj)."""
    z = lambda a, ii, jj: 0.0 if a is None else a[jj, ii]
    table = {
        (0, 0): O[j, i], (-1, 0): W[j, i], (1, 0): W[j, i + 1],
        (0, -1): S[j, i], (0, 1): S[j + 1, i],
        (-1, -1): z(SW, i, j), (1, 1): z(SW, i + 1, j + 1),
        (-1, 1): z(NW, i, j), (1, -1): z(NW, i + 1, j - 1),
    }
    return table[(di, dj)]


def matrix_from_compact(O, W, S, SW=None, NW=None) -> sp.csr_matrix:
    n = O.shape[0] - 2
    rows, cols, vals = [], [], []
    for j in range(1, n + 1):
        for i in range(1, n + 1):
            for di, dj in _DIRS:
                qi, qj = i + di, j + dj
                if 1 <= qi <= n and 1 <= qj <= n:
                    v = stencil_entry(O, W, S, SW, NW, i, j, di, dj)
                    if v != 0.0:
                        rows.append(_idx(n, i, j))
                        cols.append(_idx(n, qi, qj))
                        vals.append(v)
    return sp.coo_matrix((vals, (rows, cols)), shape=(n * n, n * n)).tocsr()


def compact_from_matrix(A: sp.spmatrix, n: int):
    """Inverse of ``matrix_from_compact`` for a symmetric 9-point matrix."""
    A = A.tocsr()
    O, W, S, SW, NW = (np.zeros((n + 2, n + 2)) for _ in range(5))
    for j in range(1, n + 1):
        for i in range(1, n + 1):
            a = _idx(n, i, j)
            O[j, i] = A[a, a]
            if i > 1:
                W[j, i] = A[a, _idx(n, i - 1, j)]
            if j > 1:
                S[j, i] = A[a, _idx(n, i, j - 1)]
            if i > 1 and j > 1:
                SW[j, i] = A[a, _idx(n, i - 1, j - 1)]
            if i > 1 and j < n:
                NW[j, i] = A[a, _idx(n, i - 1, j + 1)]
    return O, W, S, SW, NW


def prolongation(Ci: np.ndarray, nf: int) -> sp.csr_matrix:
    """Interpolation P (nf^2 x nc^2) from the eight weight planes, row by row:
    C-point (2I,2J) <- coarse (I,J) with weight 1; x-edge (2I-1,2J) <- LL from
    (I-1,J), LR from (I,J); y-edge (2I,2J-1) <- LB from (I,J-1), LA from (I,J);
    cell centre (2I-1,2J-1) <- LSW, LSE, LNW, LNE from its four corners.
    Columns of ring coarse points are dropped."""
    nc = (nf - 1) // 2
    LNE, LA, LNW, LR, LL, LSE, LB, LSW = Ci
    rows, cols, vals = [], [], []

    def put(p, I, J, w):
        if 1 <= I <= nc and 1 <= J <= nc:
            rows.append(p)
            cols.append(_idx(nc, I, J))
            vals.append(w)

    for j in range(1, nf + 1):
        for i in range(1, nf + 1):
            p = _idx(nf, i, j)
            if i % 2 == 0 and j % 2 == 0:
                put(p, i // 2, j // 2, 1.0)
            elif i % 2 == 1 and j % 2 == 0:
                I, J = (i + 1) // 2, j // 2
                put(p, I - 1, J, LL[J, I])
                put(p, I, J, LR[J, I])
            elif i % 2 == 0 and j % 2 == 1:
                I, J = i // 2, (j + 1) // 2
                put(p, I, J - 1, LB[J, I])
                put(p, I, J, LA[J, I])
            else:
                I, J = (i + 1) // 2, (j + 1) // 2
                put(p, I - 1, J - 1, LSW[J, I])
                put(p, I, J - 1, LSE[J, I])
                put(p, I - 1, J, LNW[J, I])
                put(p, I, J, LNE[J, I])
    return sp.coo_matrix((vals, (rows, cols)), shape=(nf * nf, nc * nc)).tocsr()


def colour_order(n: int) -> np.ndarray:
    """Unknowns listed colour by colour, colour(i,j) = (i mod 2) + 2 (j mod 2)."""
    order = []
    for c in range(4):
        for j in range(1, n + 1):
            for i in range(1, n + 1):
                if (i % 2) + 2 * (j % 2) == c:
                    order.append(_idx(n, i, j))
    return np.array(order)


def colour_gs(A: sp.spmatrix, b: np.ndarray, u: np.ndarray, n: int) -> np.ndarray:
    """One four-colour GS sweep: with the unknowns permuted into colour order,
    solve (D + L) u_new = b - U u_old by a dense triangular solve."""
    perm = colour_order(n)
    Ad = A.toarray()[np.ix_(perm, perm)]
    lower = np.tril(Ad)
    upper = np.triu(Ad, 1)
    rhs = b[perm] - upper @ u[perm]
    new = sla.solve_triangular(lower, rhs, lower=True)
    out = np.empty_like(u)
    out[perm] = new
    return out


def gs_matrix(A: sp.spmatrix, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Affine map of one sweep: u_new = M u_old + N b."""
    perm = colour_order(n)
    inv = np.argsort(perm)
    Ad = A.toarray()[np.ix_(perm, perm)]
    Linv = sla.solve_triangular(np.tril(Ad), np.eye(len(perm)), lower=True)
    M = -Linv @ np.triu(Ad, 1)
    Mo = M[np.ix_(inv, inv)]
    No = Linv[np.ix_(inv, inv)]
    return Mo, No


def two_grid(A, P, b, u, n, nu1, nu2):
    """Explicit two-grid cycle with an exact coarse solve of A_c = P^T A P."""
    Ad = A.toarray()
    Pd = P.toarray()
    Ac = Pd.T @ Ad @ Pd
    M, N = gs_matrix(A, n)
    for _ in range(nu1):
        u = M @ u + N @ b
    r = b - Ad @ u
    u = u + Pd @ np.linalg.solve(Ac, Pd.T @ r)
    for _ in range(nu2):
        u = M @ u + N @ b
    return u


def interior(a: np.ndarray) -> np.ndarray:
    """Padded (n+2)^2 array -> flat interior vector in unknown order."""
    return a[1:-1, 1:-1].reshape(-1)


def padded(v: np.ndarray, n: int) -> np.ndarray:
    out = np.zeros((n + 2, n + 2))
    out[1:-1, 1:-1] = v.reshape(n, n)
    return out


def line_sets(n: int):
    """Unknown index sets of the zebra line relaxation, in its order: rows
    j = 1, 3, ..., rows j = 2, 4, ..., columns i = 1, 3, ..., columns 2, 4, ..."""
    i, j = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1))
    k = (i - 1) + n * (j - 1)
    return [k[(j % 2) == 1], k[(j % 2) == 0], k[(i % 2) == 1], k[(i % 2) == 0]]


def zebra_line_gs(A: sp.spmatrix, b: np.ndarray, u: np.ndarray, n: int) -> np.ndarray:
    """u_S <- A_SS^-1 (b_S - A_S,rest u_rest) for each set S of line_sets."""
    import scipy.sparse.linalg as spla
    A = sp.csr_matrix(A)
    u = np.array(u, dtype=np.float64, copy=True)
    for S in line_sets(n):
        S = np.sort(S.reshape(-1))
        rest = np.setdiff1d(np.arange(n * n), S)
        rhs = b[S] - A[S][:, rest] @ u[rest]
        u[S] = spla.spsolve(sp.csc_matrix(A[S][:, S]), rhs)
    return u


# ------------------------------------------------- nonsymmetric operators
def matrix_from_planes(planes) -> sp.csr_matrix:
    """Matrix of nine padded planes (SW..NE): row (i,j) couples to (i+di, j+dj)
    with planes[3 (dj+1) + (di+1)][j, i]; couplings to the ring are dropped."""
    n = planes[0].shape[0] - 2
    rows, cols, vals = [], [], []
    for j in range(1, n + 1):
        for i in range(1, n + 1):
            for e, (di, dj) in enumerate(_DIRS):
                qi, qj = i + di, j + dj
                v = planes[e][j, i]
                if 1 <= qi <= n and 1 <= qj <= n and v != 0.0:
                    rows.append(_idx(n, i, j))
                    cols.append(_idx(n, qi, qj))
                    vals.append(v)
    return sp.coo_matrix((vals, (rows, cols)), shape=(n * n, n * n)).tocsr()


def planes_from_matrix(A: sp.spmatrix, n: int):
    """Inverse of ``matrix_from_planes`` for a nine-point matrix."""
    A = A.tocsr()
    out = [np.zeros((n + 2, n + 2)) for _ in range(9)]
    for j in range(1, n + 1):
        for i in range(1, n + 1):
            for e, (di, dj) in enumerate(_DIRS):
                qi, qj = i + di, j + dj
                if 1 <= qi <= n and 1 <= qj <= n:
                    out[e][j, i] = A[_idx(n, i, j), _idx(n, qi, qj)]
    return out


def two_grid_pg(A, P, R, b, u, n, nu1, nu2):
    """Explicit two-grid cycle with the Petrov-Galerkin coarse operator R A P,
    solved exactly."""
    Ad, Pd, Rd = A.toarray(), P.toarray(), R.toarray()
    Ac = Rd @ Ad @ Pd
    M, N = gs_matrix(A, n)
    for _ in range(nu1):
        u = M @ u + N @ b
    r = b - Ad @ u
    u = u + Pd @ np.linalg.solve(Ac, Rd @ r)
    for _ in range(nu2):
        u = M @ u + N @ b
    return u
