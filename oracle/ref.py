"""ctypes front-end of the C tier of the CPU oracle (test infrastructure only).

The C tier (``bmg_oracle.c``) computes the BoxMG V-cycle in FP64 (and the FP32
cycle of iterative refinement) in the paper's order of operations: Section 2
and Fig. vcycle_flowchart for the cycle, Fig. restrict_kernel for restriction,
Fig. stencil_operator for the nine-point stencil.  This module only marshals
NumPy arrays; it does no arithmetic of the method.

Array convention: level arrays are ``(n+2, n+2)`` float64, indexed ``[j, i]``
with the Dirichlet ring at 0 and n+1.  Interpolation weights are
``(8, nc+2, nc+2)`` in the plane order LNE, LA, LNW, LR, LL, LSE, LB, LSW.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None
_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)

WEIGHT_PLANES = ("LNE", "LA", "LNW", "LR", "LL", "LSE", "LB", "LSW")
FIELDS = {"O": 0, "W": 1, "S": 2, "SW": 3, "NW": 4, "Ci": 5, "u": 6, "b": 7, "r": 8}


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def lib():
    """Load (building first if the sources are newer) the oracle library."""
    global _lib
    if _lib is None:
        if _build.needs_build():
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_discretize.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.orc_discretize.restype = C.c_int
        L.orc_interp_weights.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_interp_weights.restype = C.c_int
        L.orc_rap.argtypes = [C.c_int] + [_dp] * 11
        L.orc_rap.restype = C.c_int
        L.orc_band_ldlt_factor.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
        L.orc_band_ldlt_factor.restype = C.c_int
        L.orc_band_ldlt_solve.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_band_ldlt_solve.restype = None
        L.orc_sumsq.argtypes = [C.c_int, _dp]
        L.orc_sumsq.restype = C.c_double
        for nm, p in (("orc_gs", _dp), ("orc_gs_f", _fp)):
            fn = getattr(L, nm)
            fn.argtypes = [C.c_int] + [p] * 7 + [C.c_int]
            fn.restype = None
        for nm, p in (("orc_residual", _dp), ("orc_residual_f", _fp)):
            fn = getattr(L, nm)
            fn.argtypes = [C.c_int] + [p] * 8
            fn.restype = None
        for nm, p in (("orc_restrict", _dp), ("orc_restrict_f", _fp),
                      ("orc_interp_add", _dp), ("orc_interp_add_f", _fp)):
            fn = getattr(L, nm)
            fn.argtypes = [C.c_int, p, p, p]
            fn.restype = None
        L.orc_setup.argtypes = [C.c_int, C.c_int, _dp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.orc_setup.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_destroy.restype = None
        L.orc_num_levels.argtypes = [C.c_void_p]
        L.orc_num_levels.restype = C.c_int
        L.orc_level_n.argtypes = [C.c_void_p, C.c_int]
        L.orc_level_n.restype = C.c_int
        L.orc_field.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_field.restype = _dp
        L.orc_coarse_factor.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_coarse_factor.restype = None
        L.orc_vcycle.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_vcycle.restype = None
        L.orc_step.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_step.restype = None
        L.orc_rel_residual.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_rel_residual.restype = C.c_double
        L.orc_solve.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double, C.c_int, C.c_int, _dp]
        L.orc_solve.restype = C.c_int
        L.orc_solve_ir.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double, C.c_int, _dp]
        L.orc_solve_ir.restype = C.c_int
        L.orc_make_f32.argtypes = [C.c_void_p]
        L.orc_make_f32.restype = C.c_int
        L.orc_line_factor.argtypes = [C.c_int] + [_dp] * 7
        L.orc_line_factor.restype = C.c_int
        L.orc_line_relax.argtypes = [C.c_int] + [_dp] * 11 + [C.c_int]
        L.orc_line_relax.restype = None
        L.orc_set_line_relax.argtypes = [C.c_void_p]
        L.orc_set_line_relax.restype = C.c_int
        # nonsymmetric BoxMG
        P9 = _dp * 9
        L.orc_ns_weights.argtypes = [C.c_int, P9, C.c_int, _dp]
        L.orc_ns_weights.restype = C.c_int
        L.orc_ns_rap.argtypes = [C.c_int, P9, _dp, _dp, P9]
        L.orc_ns_rap.restype = C.c_int
        L.orc_ns_gs.argtypes = [C.c_int, P9, _dp, _dp, C.c_int]
        L.orc_ns_gs.restype = None
        L.orc_ns_residual.argtypes = [C.c_int, P9, _dp, _dp, _dp]
        L.orc_ns_residual.restype = None
        L.orc_band_ldu_factor.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_band_ldu_factor.restype = C.c_int
        L.orc_band_ldu_solve.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_band_ldu_solve.restype = None
        L.orc_ns_setup.argtypes = [C.c_int, C.c_int, _dp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.orc_ns_setup.restype = C.c_void_p
        L.orc_ns_destroy.argtypes = [C.c_void_p]
        L.orc_ns_destroy.restype = None
        L.orc_ns_num_levels.argtypes = [C.c_void_p]
        L.orc_ns_num_levels.restype = C.c_int
        L.orc_ns_level_n.argtypes = [C.c_void_p, C.c_int]
        L.orc_ns_level_n.restype = C.c_int
        L.orc_ns_field.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_ns_field.restype = _dp
        L.orc_ns_coarse_factor.argtypes = [C.c_void_p, _dp, _dp, _dp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_ns_coarse_factor.restype = None
        L.orc_ns_step.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_ns_step.restype = None
        L.orc_ns_solve.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, _dp]
        L.orc_ns_solve.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray | None, dtype=np.float64):
    if a is None:
        return None
    if a.dtype != dtype or not a.flags.c_contiguous:
        raise TypeError("oracle arrays must be C-contiguous of the expected dtype")
    return a.ctypes.data_as(_dp if dtype == np.float64 else _fp)


def _c(a, dtype=np.float64):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------- helpers
def pad(a: np.ndarray) -> np.ndarray:
    """Interior ``(n, n)`` array -> ``(n+2, n+2)`` with a zero ring."""
    n = a.shape[0]
    out = np.zeros((n + 2, n + 2), dtype=a.dtype)
    out[1:-1, 1:-1] = a
    return out


def compact_from_stencil(st: np.ndarray):
    """``[n][n][K]`` stencil (K=5: S,W,O,E,N; K=9: SW,S,SE,W,O,E,NW,N,NE) ->
    padded compact planes ``(O, W, S, SW, NW)``; SW/NW are None for K=5."""
    n, _, K = st.shape
    if K == 5:
        return pad(st[:, :, 2]), pad(st[:, :, 1]), pad(st[:, :, 0]), None, None
    return (pad(st[:, :, 4]), pad(st[:, :, 3]), pad(st[:, :, 1]),
            pad(st[:, :, 0]), pad(st[:, :, 6]))


# ------------------------------------------------------------ operations
def discretize(k: np.ndarray, f: np.ndarray):
    """Five-point vertex-centred operator and right-hand side ``h^2 f``."""
    n = f.shape[0]
    k = _c(k)
    f = _c(f)
    st = np.zeros((n, n, 5))
    rhs = np.zeros((n, n))
    s = lib().orc_discretize(n, _p(k), _p(f), _p(st), _p(rhs))
    if s:
        raise OracleError(s, "discretize")
    return st, rhs


def interp_weights(O, W, S, SW=None, NW=None):
    nf = O.shape[0] - 2
    nc = (nf - 1) // 2
    Ci = np.zeros((8, nc + 2, nc + 2))
    s = lib().orc_interp_weights(nf, _p(_c(O)), _p(_c(W)), _p(_c(S)), _p(_c(SW)),
                                 _p(_c(NW)), _p(Ci))
    if s:
        raise OracleError(s, "interp_weights")
    return Ci


def rap(O, W, S, SW, NW, Ci):
    nf = O.shape[0] - 2
    nc = (nf - 1) // 2
    out = [np.zeros((nc + 2, nc + 2)) for _ in range(5)]
    s = lib().orc_rap(nf, _p(_c(O)), _p(_c(W)), _p(_c(S)), _p(_c(SW)), _p(_c(NW)),
                      _p(_c(Ci)), *[_p(o) for o in out])
    if s:
        raise OracleError(s, "rap")
    return tuple(out)


def band_of(A: np.ndarray, w: int) -> np.ndarray:
    """Lower band of a symmetric matrix in the oracle's band storage: row i holds
    A[i, k] for k = i-w .. i at column k - i + w (zeros before the first row)."""
    m = A.shape[0]
    Ab = np.zeros((m, w + 1))
    for i in range(m):
        for k in range(max(0, i - w), i + 1):
            Ab[i, k - i + w] = A[i, k]
    return Ab


def band_to_dense(Lb: np.ndarray) -> np.ndarray:
    """Unit lower triangular L from its band storage ``Lb[i, k - i + w] = L[i, k]``."""
    m, w = Lb.shape
    L = np.eye(m)
    for i in range(m):
        for k in range(max(0, i - w), i):
            L[i, k] = Lb[i, k - i + w]
    return L


def band_ldlt_factor(Ab: np.ndarray):
    """Square-root-free Cholesky of a band matrix: ``(Lb, D)`` in band storage."""
    m, w1 = Ab.shape
    w = w1 - 1
    Lb = np.zeros((m, w))
    D = np.zeros(m)
    s = lib().orc_band_ldlt_factor(m, w, _p(_c(Ab)), _p(Lb), _p(D))
    if s:
        raise OracleError(s, "band_ldlt_factor")
    return Lb, D


def band_ldlt_solve(Lb, D, b):
    m, w = Lb.shape
    x = np.zeros(m)
    lib().orc_band_ldlt_solve(m, w, _p(_c(Lb)), _p(_c(D)), _p(_c(b)), _p(x))
    return x


def ldlt_factor(A: np.ndarray):
    """Factor of a dense SPD matrix (the band routine with w = m - 1):
    ``(L, D)`` with L unit lower triangular."""
    m = A.shape[0]
    Lb, D = band_ldlt_factor(band_of(A, max(m - 1, 1)))
    return band_to_dense(Lb), D


def ldlt_solve(L, D, b):
    m = L.shape[0]
    w = max(m - 1, 1)
    Lb = np.zeros((m, w))
    for i in range(m):
        for k in range(max(0, i - w), i):
            Lb[i, k - i + w] = L[i, k]
    return band_ldlt_solve(Lb, D, b)


def line_factor(O, W, S):
    """Factors of every x-line and y-line of a level: ``(lx, rx, ly, ry)``,
    the multipliers and reciprocal pivots of each line's tridiagonal matrix at
    its grid points."""
    n = O.shape[0] - 2
    out = [np.zeros((n + 2, n + 2)) for _ in range(4)]
    s = lib().orc_line_factor(n, _p(_c(O)), _p(_c(W)), _p(_c(S)), *[_p(o) for o in out])
    if s:
        raise OracleError(s, "line_factor")
    return tuple(out)


def line_relax(O, W, S, SW, NW, factors, b, u, sweeps=1):
    """Alternating zebra line Gauss-Seidel sweeps; returns the updated copy of u."""
    n = O.shape[0] - 2
    u = np.array(u, dtype=np.float64, copy=True)
    lib().orc_line_relax(n, *[_p(_c(a)) for a in (O, W, S, SW, NW)], *[_p(_c(f)) for f in factors],
                         _p(_c(b)), _p(u), sweeps)
    return u


def sumsq(r: np.ndarray) -> float:
    """Accurately rounded sum of squares over the interior of a padded array."""
    return lib().orc_sumsq(r.shape[0] - 2, _p(_c(r)))


def gs(O, W, S, SW, NW, b, u, sweeps=1, dtype=np.float64):
    """Four-colour Gauss-Seidel sweeps; returns the updated copy of ``u``."""
    u = np.array(u, dtype=dtype, copy=True)
    fn = lib().orc_gs if dtype == np.float64 else lib().orc_gs_f
    fn(O.shape[0] - 2, *[_p(_c(a, dtype), dtype) for a in (O, W, S, SW, NW, b)],
       _p(u, dtype), sweeps)
    return u


def residual(O, W, S, SW, NW, b, u, dtype=np.float64):
    r = np.zeros_like(np.asarray(u, dtype=dtype))
    fn = lib().orc_residual if dtype == np.float64 else lib().orc_residual_f
    fn(O.shape[0] - 2, *[_p(_c(a, dtype), dtype) for a in (O, W, S, SW, NW, b, u)],
       _p(r, dtype))
    return r


def restrict(Ci, r, dtype=np.float64):
    nf = r.shape[0] - 2
    nc = (nf - 1) // 2
    bc = np.zeros((nc + 2, nc + 2), dtype=dtype)
    fn = lib().orc_restrict if dtype == np.float64 else lib().orc_restrict_f
    fn(nf, _p(_c(Ci, dtype), dtype), _p(_c(r, dtype), dtype), _p(bc, dtype))
    return bc


def interp_add(Ci, ec, u, dtype=np.float64):
    u = np.array(u, dtype=dtype, copy=True)
    fn = lib().orc_interp_add if dtype == np.float64 else lib().orc_interp_add_f
    fn(u.shape[0] - 2, _p(_c(Ci, dtype), dtype), _p(_c(ec, dtype), dtype), _p(u, dtype))
    return u


# ------------------------------------------------------------- hierarchy
class Hierarchy:
    """FP64 BoxMG hierarchy built from a ``[n][n][K]`` stencil."""

    def __init__(self, stencil: np.ndarray, nu1: int = 2, nu2: int = 1, smoother: str = "point",
                 coarsest: int = 3):
        st = _c(stencil)
        n, _, K = st.shape
        status = C.c_int(0)
        h = lib().orc_setup(n, K, _p(st), nu1, nu2, coarsest, C.byref(status))
        if not h:
            raise OracleError(status.value, "setup")
        self._h = h
        if smoother == "line":
            s = lib().orc_set_line_relax(h)
            if s:
                self.close()
                raise OracleError(s, "line factor")
        elif smoother != "point":
            raise ValueError(smoother)
        self.n = n
        self.K = K
        self.nu1, self.nu2 = nu1, nu2
        self.nlev = lib().orc_num_levels(h)
        self.xl = None

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_n(self, l: int) -> int:
        return lib().orc_level_n(self._h, l)

    def field(self, l: int, name: str) -> np.ndarray | None:
        """Copy of a level array (O, W, S, SW, NW, Ci, u, b, r)."""
        ptr = lib().orc_field(self._h, l, FIELDS[name])
        if not ptr:
            return None
        n = self.level_n(l)
        if name == "Ci":
            nc = self.level_n(l + 1)
            shape = (8, nc + 2, nc + 2)
        else:
            shape = (n + 2, n + 2)
        return np.ctypeslib.as_array(ptr, shape=shape).copy()

    def set_field(self, l: int, name: str, value: np.ndarray) -> None:
        ptr = lib().orc_field(self._h, l, FIELDS[name])
        n = self.level_n(l)
        dst = np.ctypeslib.as_array(ptr, shape=(n + 2, n + 2))
        dst[...] = value

    def op(self, l: int):
        return tuple(self.field(l, nm) for nm in ("O", "W", "S", "SW", "NW"))

    def coarse_factor(self):
        """Band factor of the coarsest level: ``(Lb, D)`` with ``Lb`` of shape
        ``(m, w)``, ``Lb[i, k - i + w] = L[i, k]`` (m = n_L^2, w = n_L + 1)."""
        m, w = C.c_int(0), C.c_int(0)
        lib().orc_coarse_factor(self._h, None, None, C.byref(m), C.byref(w))
        Lb = np.zeros((m.value, w.value))
        D = np.zeros(m.value)
        lib().orc_coarse_factor(self._h, _p(Lb), _p(D), None, None)
        return Lb, D

    def step(self, l: int, op: str, arg: int = 1) -> None:
        code = {"smooth": 0, "residual": 1, "restrict": 2, "interp": 3, "coarse": 4}[op]
        lib().orc_step(self._h, l, code, arg)

    def vcycle(self, b: np.ndarray, u: np.ndarray) -> np.ndarray:
        u = np.array(u, dtype=np.float64, copy=True)
        lib().orc_vcycle(self._h, _p(_c(b)), _p(u))
        return u

    def rel_residual(self, b, u, xl=None) -> float:
        """||b - A (u + xl)|| / ||b|| with the accurate residual."""
        return lib().orc_rel_residual(self._h, _p(_c(b)), _p(_c(u)), _p(_c(xl)))

    def solve(self, b: np.ndarray, u: np.ndarray | None = None, tol: float = 1e-10,
              max_cycles: int = 100, refine_factor: int = 16):
        """Returns ``(u, history)``; history[k] = ||b - A x^{k+1}|| / ||b||.
        Once the relative residual is <= refine_factor * tol the iterate is a
        double-FP64 pair; its low part is left in ``self.xl``."""
        u = np.zeros_like(b) if u is None else np.array(u, dtype=np.float64, copy=True)
        hist = np.zeros(max_cycles)
        self.xl = np.zeros_like(u)
        k = lib().orc_solve(self._h, _p(_c(b)), _p(u), _p(self.xl), tol, max_cycles,
                            refine_factor, _p(hist))
        if k < 0:
            raise OracleError(k, "solve")
        return u, hist[:k].copy()

    def solve_ir(self, b: np.ndarray, x: np.ndarray | None = None, tol: float = 1e-10,
                 max_iter: int = 100):
        """FP32-preconditioned refinement of a double-FP64 iterate; returns
        ``(x_high, history)`` with history[0] the initial relative residual; the
        low part is left in ``self.xl``."""
        x = np.zeros_like(b) if x is None else np.array(x, dtype=np.float64, copy=True)
        hist = np.zeros(max_iter + 1)
        self.xl = np.zeros_like(x)
        k = lib().orc_solve_ir(self._h, _p(_c(b)), _p(x), _p(self.xl), tol, max_iter, _p(hist))
        if k < 0:
            raise OracleError(k, "solve_ir")
        return x, hist[:k + 1].copy()


# ------------------------------------------------- nonsymmetric BoxMG
def _planes9(planes):
    """Nine padded planes (SW..NE) as the C array of pointers the library takes."""
    arr = [_c(a) for a in planes]
    return arr, (_dp * 9)(*[_p(a) for a in arr])


def ns_weights(planes, transpose: bool = False) -> np.ndarray:
    """Operator-induced weights of the full nine-plane operator (P), or of its
    transpose (the weights whose transpose is the restriction R)."""
    keep, A = _planes9(planes)
    nf = keep[0].shape[0] - 2
    nc = (nf - 1) // 2
    Ci = np.zeros((8, nc + 2, nc + 2))
    s = lib().orc_ns_weights(nf, A, int(transpose), _p(Ci))
    if s:
        raise OracleError(s, "ns_weights")
    return Ci


def ns_rap(planes, Pi, Ri):
    """Petrov-Galerkin coarse operator R A P as nine padded planes."""
    keep, A = _planes9(planes)
    nf = keep[0].shape[0] - 2
    nc = (nf - 1) // 2
    out = [np.zeros((nc + 2, nc + 2)) for _ in range(9)]
    _, Ac = _planes9(out)
    lib().orc_ns_rap(nf, A, _p(_c(Pi)), _p(_c(Ri)), Ac)
    return out


def ns_gs(planes, b, u, sweeps=1):
    keep, A = _planes9(planes)
    u = np.array(u, dtype=np.float64, copy=True)
    lib().orc_ns_gs(keep[0].shape[0] - 2, A, _p(_c(b)), _p(u), sweeps)
    return u


def ns_residual(planes, b, u):
    keep, A = _planes9(planes)
    r = np.zeros_like(u, dtype=np.float64)
    lib().orc_ns_residual(keep[0].shape[0] - 2, A, _p(_c(b)), _p(_c(u)), _p(r))
    return r


def band_ldu_factor(Ab: np.ndarray):
    """L D U of a band matrix in storage (m, 2w+1): returns (Lb, Ub, D)."""
    m, rw = Ab.shape
    w = (rw - 1) // 2
    Lb, Ub, D = np.zeros((m, w)), np.zeros((m, w)), np.zeros(m)
    s = lib().orc_band_ldu_factor(m, w, _p(_c(Ab)), _p(Lb), _p(Ub), _p(D))
    if s:
        raise OracleError(s, "band_ldu_factor")
    return Lb, Ub, D


def band_ldu_solve(Lb, Ub, D, b):
    m, w = Lb.shape
    x = np.zeros(m)
    lib().orc_band_ldu_solve(m, w, _p(_c(Lb)), _p(_c(Ub)), _p(_c(D)), _p(_c(b)), _p(x))
    return x


def full_planes(stencil: np.ndarray):
    """Nine padded planes (SW..NE) from a [n][n][K] stencil (K = 5: S, W, O, E,
    N; K = 9: SW..NE), zero on the ring."""
    n, _, K = stencil.shape
    out = [np.zeros((n + 2, n + 2)) for _ in range(9)]
    idx = (1, 3, 4, 5, 7) if K == 5 else tuple(range(9))
    for t, e in enumerate(idx):
        out[e][1:-1, 1:-1] = stencil[:, :, t]
    return out


NS_FIELDS = {**{f"A{e}": e for e in range(9)}, "Pi": 9, "Ri": 10, "u": 11, "b": 12, "r": 13}


class NSHierarchy:
    """Nonsymmetric BoxMG hierarchy (R = P~^T from the transposed operator,
    coarse operators R A P) of a ``[n][n][K]`` stencil."""

    def __init__(self, stencil: np.ndarray, nu1: int = 2, nu2: int = 1, coarsest: int = 3):
        st = _c(stencil)
        n, _, K = st.shape
        status = C.c_int(0)
        h = lib().orc_ns_setup(n, K, _p(st), nu1, nu2, coarsest, C.byref(status))
        if not h:
            raise OracleError(status.value, "ns_setup")
        self._h = h
        self.n = n
        self.nlev = lib().orc_ns_num_levels(h)

    def close(self):
        if self._h:
            lib().orc_ns_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_n(self, l: int) -> int:
        return lib().orc_ns_level_n(self._h, l)

    def field(self, l: int, name: str) -> np.ndarray:
        ptr = lib().orc_ns_field(self._h, l, NS_FIELDS[name])
        if not ptr:
            raise KeyError(name)
        n = self.level_n(l)
        if name in ("Pi", "Ri"):
            nc = self.level_n(l + 1)
            shape = (8, nc + 2, nc + 2)
        else:
            shape = (n + 2, n + 2)
        return np.ctypeslib.as_array(ptr, shape=shape).copy()

    def set_field(self, l: int, name: str, value: np.ndarray) -> None:
        ptr = lib().orc_ns_field(self._h, l, NS_FIELDS[name])
        n = self.level_n(l)
        np.ctypeslib.as_array(ptr, shape=(n + 2, n + 2))[...] = value

    def planes(self, l: int):
        return [self.field(l, f"A{e}") for e in range(9)]

    def coarse_factor(self):
        m, w = C.c_int(0), C.c_int(0)
        lib().orc_ns_coarse_factor(self._h, None, None, None, C.byref(m), C.byref(w))
        Lb, Ub, D = np.zeros((m.value, w.value)), np.zeros((m.value, w.value)), np.zeros(m.value)
        lib().orc_ns_coarse_factor(self._h, _p(Lb), _p(Ub), _p(D), None, None)
        return Lb, Ub, D

    def step(self, l: int, op: str, arg: int = 1) -> None:
        code = {"smooth": 0, "residual": 1, "restrict": 2, "interp": 3, "coarse": 4}[op]
        lib().orc_ns_step(self._h, l, code, arg)

    def solve(self, b: np.ndarray, u: np.ndarray | None = None, tol: float = 1e-10, max_cycles: int = 100):
        """Returns ``(u, history)``; history[k] = ||b - A u^{k+1}|| / ||b||."""
        u = np.zeros_like(b) if u is None else np.array(u, dtype=np.float64, copy=True)
        hist = np.zeros(max_cycles)
        k = lib().orc_ns_solve(self._h, _p(_c(b)), _p(u), tol, max_cycles, _p(hist))
        return u, hist[:k].copy()
