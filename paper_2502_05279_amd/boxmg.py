"""Python binding of the HIP black-box multigrid library (``include/bmg.h``).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (the workspace, inputs and outputs)
and the stream (the current torch stream at construction).  If the library is
not built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import torch

from . import build as _build

__all__ = ["BoxMGError", "Options", "Solver", "NSSolver", "solve_noalloc", "Block", "Batch", "Net", "discretize", "lib", "FIELDS", "STEPS",
           "tile_rows_set", "tile_rows_get", "solve_select", "NET_PARAMS", "NET_ARRAYS",
           "BMG_INTERP_BOXMG", "BMG_INTERP_LEARNED", "BMG_SMOOTH_POINT", "BMG_SMOOTH_LINE",
           "TRACE", "BMG_FP64", "BMG_FP32_IR", "BMG_KERNELS_BASIC", "BMG_KERNELS_FUSED"]

BMG_OK, BMG_EINVAL, BMG_EBREAKDOWN, BMG_ENOCONV, BMG_EDIVERGED, BMG_EDEVICE, BMG_EWORKSPACE = \
    0, -1, -2, -3, -4, -5, -6
BMG_FP64, BMG_FP32_IR = 0, 1
BMG_KERNELS_BASIC, BMG_KERNELS_FUSED = 0, 1
BMG_SMOOTH_POINT, BMG_SMOOTH_LINE = 0, 1
BMG_INTERP_BOXMG, BMG_INTERP_LEARNED = 0, 1
NET_PARAMS = 14184
NET_ARRAYS = {"X": 0, "H1": 1, "H2": 2, "D3": 3, "D2": 4, "D1": 5, "Y": 6}

FIELDS = {"u": 0, "b": 1, "r": 2, "O": 3, "W": 4, "S": 5, "SW": 6, "NW": 7, "Ci": 8, "LD": 9,
          "xlo": 10, "stencil": 11,
          "u32": 16, "b32": 17, "r32": 18, "O32": 19, "W32": 20, "S32": 21, "SW32": 22,
          "NW32": 23, "Ci32": 24}
STEPS = {"smooth": 0, "residual": 1, "restrict": 2, "interp": 3, "coarse": 4, "pre": 5, "post": 6}
TRACE = {"smooth": 0, "pre": 1, "post": 2, "resnorm": 3, "postpre": 4}


class Options(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int), ("max_cycles", C.c_int),
                ("precision", C.c_int), ("kernels", C.c_int), ("check_every", C.c_int),
                ("refine_factor", C.c_int), ("tile_rows", C.c_int), ("interp", C.c_int),
                ("learned_levels", C.c_int), ("net", C.c_void_p), ("smoother", C.c_int),
                ("coarsest_n", C.c_int), ("persistent_below_n", C.c_int),
                ("square_tiles_below_n", C.c_int), ("graph_mode", C.c_int)]


class Info(C.Structure):
    _fields_ = [("cycles", C.c_int), ("rel_res", C.c_double), ("rho", C.c_double),
                ("history", C.POINTER(C.c_double)), ("floor_est", C.c_double),
                ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double), ("interp_used", C.c_int),
                ("learned_levels_used", C.c_int)]


def _new_info(hist) -> Info:
    info = Info()
    info.history = C.cast(hist, C.POINTER(C.c_double))
    return info


def _info_dict(info: Info, hist, nh: int, status: int) -> dict:
    return {"cycles": info.cycles, "rel_res": info.rel_res, "rho": info.rho,
            "history": [hist[t] for t in range(nh)], "status": status, "floor_est": info.floor_est,
            "t_setup_ms": info.t_setup_ms, "t_solve_ms": info.t_solve_ms, "interp_used": info.interp_used,
            "learned_levels_used": info.learned_levels_used}


class _Handle:
    """Explicit release (``close()`` or a ``with`` block).  During interpreter
    shutdown ``__del__`` does nothing: the HIP runtime (and a profiler's hooks
    around it) may already be torn down, and a late release call into it can
    crash the process after its work is done."""

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: the module's globals may be gone by then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


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
        path = os.environ.get("BMG_LIBRARY", _build.LIB)   # a tuning variant of the same sources
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run "
                               "`python -m paper_2502_05279_amd.build` first")
        L = C.CDLL(path)
        vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
        sig = {
            "bmg_default_options": ([C.POINTER(Options)], i),
            "bmg_workspace_bytes": ([i, i, C.POINTER(Options), C.POINTER(sz)], i),
            "bmg_discretize": ([vp, vp, i, vp, vp, vp], i),
            "bmg_setup": ([C.POINTER(vp), vp, i, i, C.POINTER(Options), vp, sz, vp], i),
            "bmg_vcycle": ([vp, vp, vp, C.POINTER(d)], i),
            "bmg_solve": ([vp, vp, vp, d, C.POINTER(Info)], i),
            "bmg_solve_noalloc": ([vp, i, i, C.POINTER(Options), vp, vp, d, C.POINTER(Info), vp], i),
            "bmg_destroy": ([vp], i),
            "bmg_status_string": ([i], C.c_char_p),
            "bmg_last_error": ([], C.c_char_p),
            "bmg_num_levels": ([vp, C.POINTER(i)], i),
            "bmg_level_n": ([vp, i, C.POINTER(i)], i),
            "bmg_export": ([vp, i, i, vp], i),
            "bmg_import": ([vp, i, i, vp], i),
            "bmg_step": ([vp, i, i, i, i], i),
            "bmg_trace_enable": ([vp, i, i, i], i),
            "bmg_trace_read": ([vp, C.POINTER(i), C.POINTER(d), C.POINTER(d)], i),
            "bmg_tile_rows_set": ([i, i], i),
            "bmg_tile_rows_get": ([i, C.POINTER(i)], i),
            "bmg_batch_workspace_bytes": ([i, C.POINTER(i), C.POINTER(Options), C.POINTER(sz)], i),
            "bmg_batch_setup": ([C.POINTER(vp), i, C.POINTER(i), C.POINTER(vp), C.POINTER(Options),
                                 vp, sz, vp], i),
            "bmg_batch_solve": ([vp, C.POINTER(vp), C.POINTER(vp), d, C.POINTER(i), C.POINTER(d)], i),
            "bmg_batch_history": ([vp, i, C.POINTER(d), i, C.POINTER(i)], i),
            "bmg_batch_info": ([vp, C.POINTER(i), C.POINTER(i)], i),
            "bmg_batch_destroy": ([vp], i),
            "bmg_net_workspace_bytes": ([i, i, C.POINTER(sz)], i),
            "bmg_net_create": ([C.POINTER(vp), i, i, vp, vp, sz, vp], i),
            "bmg_net_set_params": ([vp, vp], i),
            "bmg_net_get_params": ([vp, vp], i),
            "bmg_net_destroy": ([vp], i),
            "bmg_net_forward": ([vp, i, i, vp, vp, vp, vp, vp, vp, i, sz], i),
            "bmg_net_backward": ([vp, vp, i, sz], i),
            "bmg_net_get_grad": ([vp, vp], i),
            "bmg_net_zero_grad": ([vp], i),
            "bmg_net_adam": ([vp, C.c_float, C.c_float, C.c_float, C.c_float, d], i),
            "bmg_net_export": ([vp, i, vp, C.POINTER(sz)], i),
            "bmg_net_twogrid": ([vp, vp, vp, d, i, C.POINTER(d), vp], i),
            "bmg_solve_select": ([vp, vp, vp, vp, d, i, C.POINTER(Info), C.POINTER(i), C.POINTER(d)], i),
            "bmg_block_workspace_bytes": ([vp, i, C.POINTER(sz)], i),
            "bmg_block_create": ([C.POINTER(vp), vp, i, vp, sz], i),
            "bmg_block_solve": ([vp, vp, vp, d, C.POINTER(Info), C.POINTER(i)], i),
            "bmg_block_trace_enable": ([vp, i, i, i], i),
            "bmg_block_trace_read": ([vp, C.POINTER(i), C.POINTER(d), C.POINTER(d)], i),
            "bmg_block_destroy": ([vp], i),
            "bmg_ns_workspace_bytes": ([i, i, C.POINTER(Options), C.POINTER(sz)], i),
            "bmg_ns_setup": ([C.POINTER(vp), vp, i, i, C.POINTER(Options), vp, sz, vp], i),
            "bmg_ns_solve": ([vp, vp, vp, d, C.POINTER(Info)], i),
            "bmg_ns_destroy": ([vp], i),
            "bmg_ns_num_levels": ([vp, C.POINTER(i)], i),
            "bmg_ns_level_n": ([vp, i, C.POINTER(i)], i),
            "bmg_ns_export": ([vp, i, i, vp], i),
            "bmg_ns_import": ([vp, i, i, vp], i),
            "bmg_ns_step": ([vp, i, i, i], i),
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
        if k == "net":
            o.net = None if v is None else (v.handle if isinstance(v, Net) else int(v))
        else:
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


NS_FIELDS = {**{f"A{e}": e for e in range(9)}, "Pi": 9, "Ri": 10, "u": 11, "b": 12, "r": 13, "LDU": 14}


class NSSolver(_Handle):
    """Nonsymmetric BoxMG hierarchy (restriction from the transposed operator,
    Petrov-Galerkin coarse operators) of a ``[n][n][K]`` stencil on the GPU."""

    def __init__(self, stencil: torch.Tensor, **options):
        n, n2, K = stencil.shape
        if n != n2 or K not in (5, 9):
            raise ValueError(f"stencil shape {tuple(stencil.shape)}")
        self.n = n
        self.options = default_options(**options)
        need = C.c_size_t(0)
        _check(lib().bmg_ns_workspace_bytes(n, K, C.byref(self.options), C.byref(need)), "bmg_ns_workspace_bytes")
        self.device = stencil.device
        self.workspace = torch.empty(need.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p(None)
        _check(lib().bmg_ns_setup(C.byref(h), _ptr(stencil), n, K, C.byref(self.options),
                                  self.workspace.data_ptr(), need.value, _stream()), "bmg_ns_setup")
        self._h = h
        nl = C.c_int(0)
        _check(lib().bmg_ns_num_levels(self._h, C.byref(nl)), "bmg_ns_num_levels")
        self.nlev = nl.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().bmg_ns_destroy(self._h)
            self._h = None

    def level_n(self, level: int) -> int:
        out = C.c_int(0)
        _check(lib().bmg_ns_level_n(self._h, level, C.byref(out)), "bmg_ns_level_n")
        return out.value

    def solve(self, rhs: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-10,
              raise_on_noconv: bool = True):
        if x is None:
            x = torch.zeros_like(rhs)
        hist = (C.c_double * (self.options.max_cycles + 2))()
        info = _new_info(hist)
        st = lib().bmg_ns_solve(self._h, _ptr(rhs), _ptr(x), float(tol), C.byref(info))
        if st not in (BMG_OK, BMG_ENOCONV) or (st == BMG_ENOCONV and raise_on_noconv):
            _check(st, "bmg_ns_solve")
        return x, _info_dict(info, hist, info.cycles, st)

    def export(self, level: int, field: str) -> torch.Tensor:
        f = NS_FIELDS[field]
        if f == 14:
            m = self.level_n(self.nlev - 1) ** 2
            w = self.level_n(self.nlev - 1) + 1
            out = torch.empty(2 * m * w + m, dtype=torch.float64, device=self.device)
        elif f in (9, 10):
            nc = self.level_n(level + 1)
            out = torch.empty((8, nc + 2, nc + 2), dtype=torch.float64, device=self.device)
        else:
            nl = self.level_n(level)
            out = torch.empty((nl + 2, nl + 2), dtype=torch.float64, device=self.device)
        _check(lib().bmg_ns_export(self._h, level, f, _ptr(out)), "bmg_ns_export")
        return out

    def import_(self, level: int, field: str, value: torch.Tensor) -> None:
        _check(lib().bmg_ns_import(self._h, level, NS_FIELDS[field], _ptr(value.contiguous())), "bmg_ns_import")

    def step(self, level: int, step: str, arg: int = 1) -> None:
        _check(lib().bmg_ns_step(self._h, level, STEPS[step], arg), "bmg_ns_step")


def solve_noalloc(stencil: torch.Tensor, rhs: torch.Tensor, x: torch.Tensor | None = None,
                  tol: float = 1e-10, raise_on_noconv: bool = True, **options):
    """Set-up and solve in one library call that allocates nothing (the
    hierarchy in the library's own device array, at most BMG_NOALLOC_BYTES);
    returns ``(x, info)`` as ``Solver.solve``."""
    n, n2, K = stencil.shape
    if n != n2 or K not in (5, 9) or tuple(rhs.shape) != (n, n):
        raise ValueError(f"stencil {tuple(stencil.shape)} and rhs {tuple(rhs.shape)} do not match")
    if x is None:
        x = torch.zeros_like(rhs)
    o = default_options(**options)
    hist = (C.c_double * (o.max_cycles + 2))()
    info = _new_info(hist)
    st = lib().bmg_solve_noalloc(_ptr(stencil), n, K, C.byref(o), _ptr(rhs), _ptr(x), float(tol),
                                 C.byref(info), _stream())
    if st not in (BMG_OK, BMG_ENOCONV) or (st == BMG_ENOCONV and raise_on_noconv):
        _check(st, "bmg_solve_noalloc")
    nh = info.cycles + (1 if o.precision == BMG_FP32_IR else 0)
    return x, _info_dict(info, hist, nh, st)


class Solver(_Handle):
    """BoxMG hierarchy of a ``[n][n][K]`` stencil (K = 5 or 9) on the GPU."""

    def __init__(self, stencil: torch.Tensor, workspace: torch.Tensor | None = None, **options):
        n, n2, K = stencil.shape
        if n != n2:
            raise ValueError("stencil must be [n][n][K]")
        self.n, self.kind = n, K
        self.options = default_options(**options)
        need = C.c_size_t(0)
        _check(lib().bmg_workspace_bytes(n, K, C.byref(self.options), C.byref(need)),
               "bmg_workspace_bytes")
        if workspace is not None and workspace.numel() >= need.value:
            self.workspace = workspace
        else:
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
        info = _new_info(hist)
        st = lib().bmg_solve(self._h, _ptr(rhs), _ptr(x), float(tol), C.byref(info))
        if st not in (BMG_OK, BMG_ENOCONV) or (st == BMG_ENOCONV and raise_on_noconv):
            _check(st, "bmg_solve")
        nh = info.cycles + (1 if self.options.precision == BMG_FP32_IR else 0)
        return x, _info_dict(info, hist, nh, st)

    # ------------------------------------------------------- level access
    def level_n(self, level: int) -> int:
        n = C.c_int(0)
        _check(lib().bmg_level_n(self._h, level, C.byref(n)), "bmg_level_n")
        return n.value

    def _shape(self, level: int, field: str):
        base = field[:-2] if field.endswith("32") else field
        dtype = torch.float32 if field.endswith("32") else torch.float64
        if base == "LD":
            nl = self.level_n(self.nlev - 1)
            return (nl * nl * (nl + 2),), torch.float64
        if base == "xlo":
            return (self.n + 2, self.n + 2), torch.float64
        if base == "stencil":
            n = self.level_n(level)
            return (n, n, 5 if (level == 0 and self.kind == 5) else 9), torch.float64
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
        """(launches, total ms, algorithmic bytes) of the timed launches."""
        n, ms, nb = C.c_int(0), C.c_double(0.0), C.c_double(0.0)
        _check(lib().bmg_trace_read(self._h, C.byref(n), C.byref(ms), C.byref(nb)), "bmg_trace_read")
        return n.value, ms.value, nb.value


class Block(_Handle):
    """k right-hand sides solved together on the hierarchy of ``solver`` (which
    must stay open while the block is used)."""

    def __init__(self, solver: Solver, k: int, workspace: torch.Tensor | None = None):
        self.solver, self.k, self.n = solver, k, solver.n
        need = C.c_size_t(0)
        _check(lib().bmg_block_workspace_bytes(solver._h, k, C.byref(need)), "bmg_block_workspace_bytes")
        if workspace is not None and workspace.numel() >= need.value:
            self.workspace = workspace
        else:
            self.workspace = torch.empty(need.value, dtype=torch.uint8, device=solver.device)
        b = C.c_void_p(None)
        _check(lib().bmg_block_create(C.byref(b), solver._h, k, self.workspace.data_ptr(), need.value),
               "bmg_block_create")
        self._b = b

    def close(self) -> None:
        if getattr(self, "_b", None):
            lib().bmg_block_destroy(self._b)
            self._b = None


    def solve(self, rhs: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-10,
              raise_on_noconv: bool = True):
        """rhs, x: ``[k][n][n]``.  Returns ``(x, infos)``, one dict per right-hand
        side as ``Solver.solve`` gives."""
        if rhs.shape != (self.k, self.n, self.n):
            raise ValueError(f"rhs must be [{self.k}][{self.n}][{self.n}]")
        if x is None:
            x = torch.zeros_like(rhs)
        cap = self.solver.options.max_cycles + 2
        hists = [(C.c_double * cap)() for _ in range(self.k)]
        infos = (Info * self.k)()
        for j in range(self.k):
            infos[j].history = C.cast(hists[j], C.POINTER(C.c_double))
        status = (C.c_int * self.k)()
        st = lib().bmg_block_solve(self._b, _ptr(rhs), _ptr(x), float(tol), infos, status)
        if st not in (BMG_OK, BMG_ENOCONV) or (st == BMG_ENOCONV and raise_on_noconv):
            _check(st, "bmg_block_solve")
        out = [{"cycles": infos[j].cycles, "rel_res": infos[j].rel_res, "rho": infos[j].rho,
                "history": [hists[j][t] for t in range(infos[j].cycles)], "status": status[j]}
               for j in range(self.k)]
        return x, out

    def trace_enable(self, kclass: str, level: int = 0, on: bool = True) -> None:
        _check(lib().bmg_block_trace_enable(self._b, TRACE[kclass], level, int(on)), "bmg_block_trace_enable")

    def trace_read(self):
        """(launches, total ms, algorithmic bytes) of the timed launches."""
        n, ms, nb = C.c_int(0), C.c_double(0.0), C.c_double(0.0)
        _check(lib().bmg_block_trace_read(self._b, C.byref(n), C.byref(ms), C.byref(nb)), "bmg_block_trace_read")
        return n.value, ms.value, nb.value


def tile_rows_set(n: int, rows: int) -> None:
    """Rows per tile of the fused passes on levels of size n (0 = default)."""
    _check(lib().bmg_tile_rows_set(n, rows), "bmg_tile_rows_set")


def tile_rows_get(n: int) -> int:
    r = C.c_int(0)
    _check(lib().bmg_tile_rows_get(n, C.byref(r)), "bmg_tile_rows_get")
    return r.value


class Batch(_Handle):
    """Independent problems of uneven sizes solved together (FP32 V-cycles in
    double-FP64 refinement, one persistent launch per group of steps)."""

    def __init__(self, stencils: list, **options):
        self.n = [int(s.shape[0]) for s in stencils]
        self.nprob = len(stencils)
        self.options = default_options(**options)
        nn = (C.c_int * self.nprob)(*self.n)
        need = C.c_size_t(0)
        _check(lib().bmg_batch_workspace_bytes(self.nprob, nn, C.byref(self.options),
                                               C.byref(need)), "bmg_batch_workspace_bytes")
        dev = stencils[0].device
        self.workspace = torch.empty(need.value, dtype=torch.uint8, device=dev)
        ptrs = (C.c_void_p * self.nprob)(*[_ptr(s) for s in stencils])
        h = C.c_void_p(None)
        _check(lib().bmg_batch_setup(C.byref(h), self.nprob, nn, ptrs, C.byref(self.options),
                                     self.workspace.data_ptr(), need.value, _stream()),
               "bmg_batch_setup")
        self._h = h
        self.device = dev

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().bmg_batch_destroy(self._h)
            self._h = None


    def solve(self, rhs: list, x: list | None = None, tol: float = 1e-10,
              raise_on_noconv: bool = True):
        """Returns ``(x, steps, rel_res, status)``."""
        if x is None:
            x = [torch.zeros_like(r) for r in rhs]
        rp = (C.c_void_p * self.nprob)(*[_ptr(r) for r in rhs])
        xp = (C.c_void_p * self.nprob)(*[_ptr(v) for v in x])
        steps = (C.c_int * self.nprob)()
        rel = (C.c_double * self.nprob)()
        st = lib().bmg_batch_solve(self._h, rp, xp, float(tol), steps, rel)
        if st not in (BMG_OK, BMG_ENOCONV) or (st == BMG_ENOCONV and raise_on_noconv):
            _check(st, "bmg_batch_solve")
        return x, list(steps), list(rel), st

    def history(self, p: int):
        cap = self.options.max_cycles + 2
        buf = (C.c_double * cap)()
        cnt = C.c_int(0)
        _check(lib().bmg_batch_history(self._h, p, buf, cap, C.byref(cnt)), "bmg_batch_history")
        return [buf[t] for t in range(cnt.value)]

    def info(self):
        nb, g = C.c_int(0), C.c_int(0)
        _check(lib().bmg_batch_info(self._h, C.byref(nb), C.byref(g)), "bmg_batch_info")
        return {"workgroups": nb.value, "graph": {0: "not built", 1: "replayed", 2: "refused"}[g.value]}


class Net(_Handle):
    """Learned-interpolation network on the GPU (parameters, Adam state and
    activation buffers in one workspace)."""

    def __init__(self, params, max_n: int, train: bool = True, device="cuda:0"):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size != NET_PARAMS:
            raise ValueError(f"expected {NET_PARAMS} parameters")
        need = C.c_size_t(0)
        _check(lib().bmg_net_workspace_bytes(max_n, int(train), C.byref(need)), "bmg_net_workspace_bytes")
        self.workspace = torch.empty(need.value, dtype=torch.uint8, device=device)
        h = C.c_void_p(None)
        _check(lib().bmg_net_create(C.byref(h), max_n, int(train), p.ctypes.data, self.workspace.data_ptr(),
                                    need.value, _stream()), "bmg_net_create")
        self._h = h
        self.max_n = max_n
        self.device = torch.device(device)

    @property
    def handle(self) -> int:
        return self._h.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().bmg_net_destroy(self._h)
            self._h = None


    def set_params(self, params) -> None:
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        _check(lib().bmg_net_set_params(self._h, p.ctypes.data), "bmg_net_set_params")

    def params(self):
        import numpy as np
        p = np.zeros(NET_PARAMS, dtype=np.float32)
        _check(lib().bmg_net_get_params(self._h, p.ctypes.data), "bmg_net_get_params")
        return p

    def forward(self, O, W, S, SW=None, NW=None, out: torch.Tensor | None = None) -> torch.Tensor:
        """Weight planes (8, nc+2, nc+2) of a level given as padded planes
        (into `out` if given)."""
        n = O.shape[0] - 2
        nc = (n - 1) // 2
        Ci = torch.zeros((8, nc + 2, nc + 2), dtype=torch.float64, device=O.device) if out is None else out
        _check(lib().bmg_net_forward(self._h, n, n + 2, _ptr(O), _ptr(W), _ptr(S), _ptr(SW), _ptr(NW),
                                     _ptr(Ci), nc + 2, (nc + 2) * (nc + 2)), "bmg_net_forward")
        return Ci

    def backward(self, dCi: torch.Tensor) -> None:
        nc = dCi.shape[1] - 2
        _check(lib().bmg_net_backward(self._h, _ptr(dCi), nc + 2, (nc + 2) * (nc + 2)), "bmg_net_backward")

    def grad(self):
        import numpy as np
        g = np.zeros(NET_PARAMS)
        _check(lib().bmg_net_get_grad(self._h, g.ctypes.data), "bmg_net_get_grad")
        return g

    def zero_grad(self) -> None:
        _check(lib().bmg_net_zero_grad(self._h), "bmg_net_zero_grad")

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             scale: float = 1.0) -> None:
        _check(lib().bmg_net_adam(self._h, lr, beta1, beta2, eps, scale), "bmg_net_adam")

    def export(self, what: str) -> torch.Tensor:
        """An activation or gradient array as bfloat16 bits (int16 tensor,
        points x channels)."""
        nbytes = C.c_size_t(0)
        _check(lib().bmg_net_export(self._h, NET_ARRAYS[what], None, C.byref(nbytes)), "bmg_net_export")
        out = torch.empty(nbytes.value // 2, dtype=torch.int16, device=self.device)
        _check(lib().bmg_net_export(self._h, NET_ARRAYS[what], out.data_ptr(), C.byref(nbytes)),
               "bmg_net_export")
        return out

    def twogrid(self, solver: "Solver", r0: torch.Tensor, inner_tol: float = 1e-8, inner_max: int = 30,
                want_grad_planes: bool = False):
        """One training sample; returns (loss, dL/dCi or None)."""
        loss = C.c_double(0.0)
        d = None
        if want_grad_planes:
            nc = solver.level_n(1)
            d = torch.zeros((8, nc + 2, nc + 2), dtype=torch.float64, device=r0.device)
        _check(lib().bmg_net_twogrid(self._h, solver._h, _ptr(r0), float(inner_tol), int(inner_max),
                                     C.byref(loss), _ptr(d) if d is not None else None), "bmg_net_twogrid")
        return loss.value, d


def solve_select(learned: Solver, boxmg: Solver, rhs: torch.Tensor, x: torch.Tensor | None = None,
                 tol: float = 1e-10, probe_cycles: int = 8, raise_on_noconv: bool = True):
    """Probe both hierarchies (probe_cycles V-cycles each), continue with the
    one whose factor over the probe's second half is smaller (a learned
    hierarchy is watched every 16 cycles and hands over to BoxMG if it falls
    behind); returns (x, info, used, (rho_learned, rho_boxmg)), info with the
    total cycles, the final relative residual and the last call's rho."""
    if x is None:
        x = torch.zeros_like(rhs)
    cap = max(learned.options.max_cycles, boxmg.options.max_cycles) + 2
    hist = (C.c_double * cap)()
    info = _new_info(hist)
    used = C.c_int(0)
    rho = (C.c_double * 2)()
    st = lib().bmg_solve_select(learned._h, boxmg._h, _ptr(rhs), _ptr(x), float(tol), int(probe_cycles),
                                C.byref(info), C.byref(used), rho)
    if st not in (BMG_OK, BMG_ENOCONV) or (st == BMG_ENOCONV and raise_on_noconv):
        _check(st, "bmg_solve_select")
    nh = max(0, info.cycles - int(probe_cycles))
    out = _info_dict(info, hist, min(nh, cap), st)
    return x, out, used.value, (rho[0], rho[1])
