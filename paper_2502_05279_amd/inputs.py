"""Seeded synthetic inputs for the BoxMG workloads.

This module holds only random-number draws and array reshaping: no step of
the multigrid method (discretisation, setup, cycling) lives here, so that the
CPU oracle and the HIP path can both be fed from it without sharing any of the
method's arithmetic.

Conventions (shared by every consumer):

* interior grid ``n x n`` with ``n = 2**m - 1`` vertices per side, mesh width
  ``h = 1/(n+1)``;
* cell coefficients ``k`` have shape ``(n+1, n+1)`` and are indexed
  ``k[jc, ic]``; cell ``(ic, jc)`` has the four vertices ``(ic..ic+1, jc..jc+1)``;
* the source ``f`` has shape ``(n, n)`` and is indexed ``f[j-1, i-1]`` for the
  interior vertex ``(i, j)``;
* arrays are C-ordered: rows run over ``j`` (north), columns over ``i`` (east).

Every array comes from its own ``numpy.random.default_rng(seed)`` (PCG64) in
C order, so a given seed always produces the same bytes.

The workloads follow the model problem ``-div(k grad u) = f`` with
homogeneous Dirichlet boundaries (Section 2, Eq. 1 of the paper); the
coefficient fields (constant, block-wise jumping, per-cell log-normal) are the
synthetic stand-ins the workloads are defined on.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Problem",
    "uniform_source",
    "constant_k",
    "blocked_log10_k",
    "lognormal_k",
    "poisson_127",
    "jumping_4095",
    "jumping_8191",
    "jumping",
    "batch_512",
    "learned_train_field",
    "NET_SHAPES",
    "NET_SIZE",
    "net_init",
    "net_random",
    "residual_probe",
    "learned_eval_4095",
]


@dataclass
class Problem:
    """One seeded problem instance: cell coefficients ``k`` and source ``f``."""

    n: int
    k: np.ndarray  # (n+1, n+1) float64, k[jc, ic]
    f: np.ndarray  # (n, n) float64, f[j-1, i-1]
    name: str = ""


def _check_n(n: int) -> None:
    if n < 3 or (n + 1) & n:
        raise ValueError(f"interior size must be 2**m - 1 with m >= 2, got {n}")


def uniform_source(n: int, seed: int) -> np.ndarray:
    """``f ~ U[-1, 1]`` i.i.d. per interior vertex, shape ``(n, n)``."""
    _check_n(n)
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, n))


def constant_k(n: int, value: float = 1.0) -> np.ndarray:
    _check_n(n)
    return np.full((n + 1, n + 1), float(value))


def blocked_log10_k(n: int, block: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Piecewise-constant ``k`` on square blocks of ``block x block`` cells.

    One independent ``log10 k ~ U[lo, hi]`` is drawn per block (block array in
    C order), then each block value is repeated over its cells.
    """
    _check_n(n)
    cells = n + 1
    if cells % block:
        raise ValueError(f"block {block} does not tile {cells} cells")
    nb = cells // block
    logk = np.random.default_rng(seed).uniform(lo, hi, size=(nb, nb))
    logk = np.repeat(np.repeat(logk, block, axis=0), block, axis=1)
    return np.power(10.0, logk)


def lognormal_k(n: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """``ln k ~ N(0, sigma^2)`` i.i.d. per cell, drawn from ``rng``."""
    _check_n(n)
    return np.exp(rng.normal(0.0, sigma, size=(n + 1, n + 1)))


# --- the named workloads --------------------------------------------------

def poisson_127(seed_f: int = 101) -> Problem:
    """Constant-coefficient Poisson, 127x127 interior, ``k = 1``."""
    n = 127
    return Problem(n, constant_k(n), uniform_source(n, seed_f), "poisson_127")


def jumping(n: int, block: int, lo: float, hi: float, seed_k: int, seed_f: int,
            name: str = "") -> Problem:
    """Block-wise jumping coefficients with ``log10 k ~ U[lo, hi]`` per block."""
    return Problem(n, blocked_log10_k(n, block, lo, hi, seed_k),
                   uniform_source(n, seed_f), name or f"jumping_{n}")


def jumping_4095(seed_k: int = 201, seed_f: int = 202, n: int = 4095) -> Problem:
    """4095^2 interior, 64x64-cell blocks, ``log10 k ~ U[-4, 4]``.

    ``n`` may be lowered (keeping the 64-cell block size) for quick cases.
    """
    return jumping(n, 64, -4.0, 4.0, seed_k, seed_f, f"jumping_{n}_c1e8")


def extra_sources(n: int, k: int, seed0: int = 202):
    """k right-hand-side fields on one operator: ``f_j ~ U[-1, 1]`` drawn with
    seed ``seed0 + j`` (so f_0 is the single-problem workload's own source)."""
    return [uniform_source(n, seed0 + j) for j in range(k)]


def jumping_8191(seed_k: int = 301, seed_f: int = 302, n: int = 8191) -> Problem:
    """8191^2 interior, 128x128-cell blocks, ``log10 k ~ U[-3, 3]``."""
    return jumping(n, 128, -3.0, 3.0, seed_k, seed_f, f"jumping_{n}_c1e6")


def batch_512(count: int = 512, m_lo: int = 6, m_hi: int = 10, sigma: float = 1.5,
              seed: int = 401) -> list[Problem]:
    """Independent problems of uneven size from one generator.

    Draw order: the array of exponents ``m ~ U{m_lo..m_hi}`` first, then for each
    problem in order its ``k`` (per-cell log-normal) and then its ``f``.
    """
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    out = []
    for idx, m in enumerate(ms):
        n = (1 << int(m)) - 1
        k = lognormal_k(n, sigma, rng)
        f = rng.uniform(-1.0, 1.0, size=(n, n))
        out.append(Problem(n, k, f, f"batch_{idx}_n{n}"))
    return out


def learned_train_field(seed: int, n: int = 255, block: int = 16,
                        lo: float = -4.0, hi: float = 4.0) -> Problem:
    """A training coefficient field for the learned interpolation."""
    return jumping(n, block, lo, hi, seed, seed + 7_000_000, f"train_{seed}")


# ------------------------------------------------------ learned interpolation
# Shapes of the network parameters, in the order of the flat parameter vector:
# conv1 weights [tap][in][out], bias, conv2 weights and bias, conv3 weights and
# bias.  A tap t = 3 (dy + 1) + (dx + 1) reads the point offset by (dx, dy).
NET_SHAPES = (("W1", (9, 9, 32)), ("b1", (32,)), ("W2", (9, 32, 32)), ("b2", (32,)),
              ("W3", (9, 32, 8)), ("b3", (8,)))
NET_SIZE = sum(int(np.prod(s)) for _, s in NET_SHAPES)


def net_init(seed: int = 501) -> np.ndarray:
    """Initial flat parameter vector (float32): weights of the first two layers
    uniform in +-sqrt(6 / fan_in) (fan_in = 9 taps x input channels), the
    output layer's weights and every bias zero, so that training starts from
    corrections of zero."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shape in NET_SHAPES:
        if name == "W3":
            out.append(np.zeros(shape).ravel())
        elif name.startswith("W"):
            bound = np.sqrt(6.0 / (shape[0] * shape[1]))
            out.append(rng.uniform(-bound, bound, size=shape).ravel())
        else:
            out.append(np.zeros(shape).ravel())
    return np.concatenate(out).astype(np.float32)


def net_random(seed: int, bias_scale: float = 0.1) -> np.ndarray:
    """A random parameter vector with non-zero biases, for parity tests."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shape in NET_SHAPES:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / (shape[0] * shape[1]))
            out.append(rng.uniform(-bound, bound, size=shape).ravel())
        else:
            out.append(rng.uniform(-bias_scale, bias_scale, size=shape).ravel())
    return np.concatenate(out).astype(np.float32)


def residual_probe(n: int, seed: int) -> np.ndarray:
    """Random initial residual r0 of a two-grid training sample, uniform[-1,1]
    on the n x n interior."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, n))


def learned_eval_4095(seed_k: int = 601, seed_f: int = 602, n: int = 4095, block: int = 16) -> Problem:
    """Evaluation field of the learned interpolation: contrast 1e6 (log10 k
    uniform in [-3, 3]) on blocks of the training fields' size."""
    return jumping(n, block, -3.0, 3.0, seed_k, seed_f, f"learned_eval_{n}")


# ----------------------------------------------------- nonsymmetric operators
def upwind_convection(n: int, beta: float, flow: str = "rotating") -> np.ndarray:
    """The convection part of a convection-diffusion test operator, as a
    [n][n][5] stencil (S, W, O, E, N) to add to the diffusion stencil: the
    first-order upwind difference of b . grad u on the vertex grid, scaled
    like the diffusion operator (times h^2, so h |b| per direction), which
    keeps the sum an M-matrix.  Velocity at vertex (x, y) = (i h, j h):
    "rotating": b = beta (-sin(pi x) cos(pi y), cos(pi x) sin(pi y)) (a
    recirculating cell); "constant": b = beta (cos 0.4, sin 0.4).  Couplings
    to the Dirichlet boundary are dropped from the off-diagonal entries and
    kept in the centre, as in the diffusion stencil."""
    _check_n(n)
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    X, Y = np.meshgrid(x, x)                           # [j][i]
    if flow == "rotating":
        bx = -beta * np.sin(np.pi * X) * np.cos(np.pi * Y)
        by = beta * np.cos(np.pi * X) * np.sin(np.pi * Y)
    elif flow == "constant":
        bx = np.full((n, n), beta * np.cos(0.4))
        by = np.full((n, n), beta * np.sin(0.4))
    else:
        raise ValueError(flow)
    st = np.zeros((n, n, 5))
    st[:, :, 1] = -h * np.maximum(bx, 0.0)            # W: upwind side for bx > 0
    st[:, :, 3] = -h * np.maximum(-bx, 0.0)           # E
    st[:, :, 0] = -h * np.maximum(by, 0.0)            # S
    st[:, :, 4] = -h * np.maximum(-by, 0.0)           # N
    st[:, :, 2] = h * (np.abs(bx) + np.abs(by))       # O
    st[:, 0, 1] = st[0, :, 0] = st[:, -1, 3] = st[-1, :, 4] = 0.0
    return st
