"""Python binding of the HIP black-box multigrid library (``include/bmg.h``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (the workspace, inputs and outputs)
and the stream (the current torch stream at construction).  If the library is
not built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

from . import build as _build

__all__ = ["BoxMGError", "Options", "Solver", "discretize", "lib", "FIELDS", "STEPS",
           "TRACE", "BMG_FP64", "BMG_FP32_IR", "BMG_KERNELS_BASIC", "BMG_KERNELS_FUSED"]

BMG_OK, BMG_EINVAL, BMG_EBREAKDOWN, BMG_ENOCONV, BMG_EDIVERGED, BMG_EDEVICE, BMG_EWORKSPACE = \
    0, -1, -2, -3, -4, -5, -6
BMG_FP64, BMG_FP32_IR = 0, 1
BMG_KERNELS_BASIC, BMG_KERNELS_FUSED = 0, 1

FIELDS = {"u": 0, "b": 1, "r": 2, "O": 3, "W": 4, "S": 5, "SW": 6, "NW": 7, "Ci": 8, "LD": 9,
          "xlo": 10,
          "u32": 16, "b32": 17, "r32": 18, "O32": 19, "W32": 20, "S32": 21, "SW32": 22,
          "NW32": 23, "Ci32": 24}
STEPS = {"smooth": 0, "residual": 1, "restrict": 2, "interp": 3, "coarse": 4, "pre": 5, "post": 6}
TRACE = {"smooth": 0, "pre": 1, "post": 2, "resnorm": 3}


class Options(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int), ("max_cycles", C.c_int),
                ("precision", C.c_int), ("kernels", C.c_int), ("check_every", C.c_int),
                ("refine_factor", C.c_int), ("tile_rows", C.c_int), ("reserved", C.c_int * 8)]


class Info(C.Structure):
    _fields_ = [("cycles", C.c_int), ("rel_res", C.c_double), ("rho", C.c_double),
                ("history", C.POINTER(C.c_double))]


class BoxMGError(RuntimeError):
    def __init__(self, status: int, call: str, detail: str):
        super().__init__(f"{call}: status {status}: {detail}")
        self.status = status
        self.detail = detail


_lib = None


def lib():
    """The loaded ``libbmg.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"{_build.LIB} is not built; run "
                               "`python -m paper_2502_05279_amd.build` first")
        L = C.CDLL(_build.LIB)
        vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
        sig = {
            "bmg_default_options": ([C.POINTER(Options)], i),
            "bmg_workspace_bytes": ([i, i, C.POINTER(Options), C.POINTER(sz)], i),
            "bmg_discretize": ([vp, vp, i, vp, vp, vp], i),
            "bmg_setup": ([C.POINTER(vp), vp, i, i, C.POINTER(Options), vp, sz, vp], i),
            "bmg_vcycle": ([vp, vp, vp, C.POINTER(d)], i),
            "bmg_solve": ([vp, vp, vp, d, C.POINTER(Info)], i),
            "bmg_destroy": ([vp], i),
            "bmg_status_string": ([i], C.c_char_p),
            "bmg_last_error": ([], C.c_char_p),
            "bmg_num_levels": ([vp, C.POINTER(i)], i),
            "bmg_level_n": ([vp, i, C.POINTER(i)], i),
            "bmg_export": ([vp, i, i, vp], i),
            "bmg_import": ([vp, i, i, vp], i),
            "bmg_step": ([vp, i, i, i, i], i),
            "bmg_trace_enable": ([vp, i, i, i], i),
            "bmg_trace_read": ([vp, C.POINTER(i), C.POINTER(d)], i),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status: int, call: str) -> None:
    if status != BMG_OK:
        raise BoxMGError(status, call, lib().bmg_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None, dtype=torch.float64) -> int | None:
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor, got {t.dtype} "
                        f"{t.device} contiguous={t.is_contiguous()}")
    return t.data_ptr()


def default_options(**kw) -> Options:
    o = Options()
    _check(lib().bmg_default_options(C.byref(o)), "bmg_default_options")
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, int(v))
    return o


def workspace_bytes(n: int, kind: int = 5, **opts) -> int:
    o = default_options(**opts)
    out = C.c_size_t(0)
    _check(lib().bmg_workspace_bytes(n, kind, C.byref(o), C.byref(out)), "bmg_workspace_bytes")
    return out.value


def discretize(k: torch.Tensor, f: torch.Tensor):
    """Five-point vertex-centred operator ``[n][n][5]`` (S, W, O, E, N) and
    right-hand side ``h^2 f`` from cell coefficients ``k`` (n+1)^2 and source f."""
    n = f.shape[0]
    st = torch.empty((n, n, 5), dtype=torch.float64, device=f.device)
    rhs = torch.empty((n, n), dtype=torch.float64, device=f.device)
    _check(lib().bmg_discretize(_ptr(k), _ptr(f), n, _ptr(st), _ptr(rhs), _stream()),
           "bmg_discretize")
    return st, rhs


class Solver:
    """BoxMG hierarchy of a ``[n][n][K]`` stencil (K = 5 or 9) on the GPU."""

    def __init__(self, stencil: torch.Tensor, **options):
        n, n2, K = stencil.shape
        if n != n2:
            raise ValueError("stencil must be [n][n][K]")
        self.n, self.kind = n, K
        self.options = default_options(**options)
        need = C.c_size_t(0)
        _check(lib().bmg_workspace_bytes(n, K, C.byref(self.options), C.byref(need)),
               "bmg_workspace_bytes")
        self.workspace = torch.empty(need.value, dtype=torch.uint8, device=stencil.device)
        h = C.c_void_p(None)
        _check(lib().bmg_setup(C.byref(h), _ptr(stencil), n, K, C.byref(self.options),
                               self.workspace.data_ptr(), need.value, _stream()), "bmg_setup")
        self._h = h
        nl = C.c_int(0)
        _check(lib().bmg_num_levels(h, C.byref(nl)), "bmg_num_levels")
        self.nlev = nl.value
        self.device = stencil.device

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().bmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- solves
    def vcycle(self, rhs: torch.Tensor, x: torch.Tensor, want_residual: bool = True):
        rel = C.c_double(0.0)
        _check(lib().bmg_vcycle(self._h, _ptr(rhs), _ptr(x),
                                C.byref(rel) if want_residual else None), "bmg_vcycle")
        return rel.value if want_residual else None

    def solve(self, rhs: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-10,
              raise_on_noconv: bool = True):
        """Returns ``(x, info)``; info has cycles, rel_res, rho, history, status."""
        if x is None:
            x = torch.zeros_like(rhs)
        hist = (C.c_double * (self.options.max_cycles + 2))()
        info = Info(0, 0.0, 0.0, C.cast(hist, C.POINTER(C.c_double)))
        st = lib().bmg_solve(self._h, _ptr(rhs), _ptr(x), float(tol), C.byref(info))
        if st not in (BMG_OK, BMG_ENOCONV) or (st == BMG_ENOCONV and raise_on_noconv):
            _check(st, "bmg_solve")
        nh = info.cycles + (1 if self.options.precision == BMG_FP32_IR else 0)
        out = {"cycles": info.cycles, "rel_res": info.rel_res, "rho": info.rho,
               "history": [hist[t] for t in range(nh)], "status": st}
        return x, out

    # ------------------------------------------------------- level access
    def level_n(self, level: int) -> int:
        n = C.c_int(0)
        _check(lib().bmg_level_n(self._h, level, C.byref(n)), "bmg_level_n")
        return n.value

    def _shape(self, level: int, field: str):
        base = field[:-2] if field.endswith("32") else field
        dtype = torch.float32 if field.endswith("32") else torch.float64
        if base == "LD":
            return (90,), torch.float64
        if base == "xlo":
            return (self.n + 2, self.n + 2), torch.float64
        if base == "Ci":
            nc = self.level_n(level + 1)
            return (8, nc + 2, nc + 2), dtype
        n = self.level_n(level)
        return (n + 2, n + 2), dtype

    def export(self, level: int, field: str) -> torch.Tensor:
        shape, dtype = self._shape(level, field)
        out = torch.empty(shape, dtype=dtype, device=self.device)
        _check(lib().bmg_export(self._h, level, FIELDS[field], _ptr(out, dtype)), "bmg_export")
        return out

    def import_(self, level: int, field: str, value: torch.Tensor) -> None:
        shape, dtype = self._shape(level, field)
        if tuple(value.shape) != shape:
            raise ValueError(f"{field} on level {level} has shape {shape}")
        _check(lib().bmg_import(self._h, level, FIELDS[field], _ptr(value, dtype)), "bmg_import")

    def step(self, level: int, step: str, arg: int = 1, fp32: bool = False) -> None:
        _check(lib().bmg_step(self._h, level, STEPS[step], arg, int(fp32)), "bmg_step")

    # ------------------------------------------------------------ tracing
    def trace_enable(self, kclass: str, level: int = 0, on: bool = True) -> None:
        _check(lib().bmg_trace_enable(self._h, TRACE[kclass], level, int(on)), "bmg_trace_enable")

    def trace_read(self):
        n, ms = C.c_int(0), C.c_double(0.0)
        _check(lib().bmg_trace_read(self._h, C.byref(n), C.byref(ms)), "bmg_trace_read")
        return n.value, ms.value
