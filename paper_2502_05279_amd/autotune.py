"""Tile-shape autotuner of the fused passes.

For each level size n it times the fused pre and post passes for a set of
candidate tile heights (rows per workgroup tile) with the library's HIP-event
trace, on a five-point level (the fine level of an n x n problem) and on a
nine-point level (level 1 of a (2n+1) x (2n+1) problem), picks the fastest
and installs it with ``bmg_tile_rows_set``.  Results are cached in a JSON
file keyed by architecture, precision and n.
"""
from __future__ import annotations

import json
import os

import torch

from . import boxmg, inputs

DEFAULT_CANDIDATES = (2, 4, 8, 16, 32, 64, 128)

# timings (ms per pre+post pass pair, by tile height) of the last tune() call
LAST: dict = {}


def _cache_path() -> str:
    return os.environ.get("BMG_TUNE_CACHE",
                          os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib",
                                       "tile_rows.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "gfx950"


def _time_level(stencil, rhs, level: int, rows: int, precision: int, cycles: int) -> float:
    S = boxmg.Solver(stencil, tile_rows=rows, precision=precision)
    x = torch.zeros_like(rhs)
    S.vcycle(rhs, x, want_residual=False)
    total = 0.0
    for cls in ("pre", "post"):
        S.trace_enable(cls, level)
        for _ in range(cycles):
            S.vcycle(rhs, x, want_residual=False)
        nl, ms, _ = S.trace_read()
        S.trace_enable(cls, level, on=False)
        total += ms / max(nl, 1)
    S.close()
    return total


def tune(sizes=(127, 255, 511, 1023, 2047), precision: int = boxmg.BMG_FP64,
         candidates=DEFAULT_CANDIDATES, cycles: int = 5, use_cache: bool = True,
         verbose: bool = False) -> dict:
    """Returns {n: rows} and installs it in the library's tile table."""
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    dev = torch.device("cuda:0")
    out = {}
    for n in sizes:
        key = f"{_arch()}:{'fp32' if precision == boxmg.BMG_FP32_IR else 'fp64'}:{n}"
        if key in cache:
            out[n] = int(cache[key]["rows"])
            LAST[n] = cache[key]["ms"]
            boxmg.tile_rows_set(n, out[n])
            continue
        timings = {}
        probs = [(inputs.jumping(n, max(2, (n + 1) // 16), -2, 2, 7, 8), 0)]
        if 2 * n + 1 <= 4095:
            probs.append((inputs.jumping(2 * n + 1, max(2, (2 * n + 2) // 16), -2, 2, 7, 8), 1))
        for rows in candidates:
            t = 0.0
            for p, level in probs:
                st, rhs = boxmg.discretize(torch.from_numpy(p.k).to(dev), torch.from_numpy(p.f).to(dev))
                t += _time_level(st, rhs, level, rows, precision, cycles)
            timings[rows] = t
        best = min(timings, key=timings.get)
        out[n] = best
        cache[key] = {"rows": best, "ms": timings}
        LAST[n] = timings
        boxmg.tile_rows_set(n, best)
        if verbose:
            print(f"tile rows n={n}: " + ", ".join(f"{r}:{t * 1e3:.0f}us" for r, t in timings.items())
                  + f" -> {best}", flush=True)
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return out


def tune_batch(run, sizes, candidates=(16, 32, 64), verbose: bool = False) -> dict:
    """Tile height for a batch: in a batch every problem's passes share the
    chip, so the objective is the whole batched solve rather than one level's
    passes.  ``run()`` performs one timed batched solve and returns its seconds;
    each candidate height is installed for every size, the fastest is kept.
    Returns {n: rows}; the timings (ms) go to ``LAST["batch"]``."""
    timings = {}
    for rows in candidates:
        for n in sizes:
            boxmg.tile_rows_set(n, rows)
        timings[rows] = run() * 1e3
        if verbose:
            print(f"batch tile rows {rows}: {timings[rows]:.1f} ms", flush=True)
    best = min(timings, key=timings.get)
    for n in sizes:
        boxmg.tile_rows_set(n, best)
    LAST["batch"] = timings
    return {n: best for n in sizes}
