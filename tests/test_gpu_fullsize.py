"""Parity at the workloads' full sizes, in the launch configuration bench.py
times: default options, hence the default tile heights of the large levels
and the weights computed in the fine pre pass.  Whole levels are compared
element by element; the oracle's C tier finishes a 4095^2 set-up in seconds.
The inputs are the benchmark's own (the 4095^2 jumping-coefficient field and
its source, and for the FP32 refinement the 8191^2 field)."""
import numpy as np
import pytest
import torch

from oracle import ref
from paper_2502_05279_amd import boxmg, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def same(a, b, what=""):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    bad = ~(a == b)
    assert not bad.any(), f"{what}: {bad.sum()} of {a.size} differ; first at " \
                          f"{np.argwhere(bad)[0]}: {a[bad][0]!r} vs {b[bad][0]!r}"


def rand_level(rng, n, dtype=np.float64):
    a = np.zeros((n + 2, n + 2))
    a[1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(n, n))
    return a.astype(dtype)


@pytest.fixture(scope="module")
def jumping4095():
    p = inputs.jumping_4095()
    kk = dev(p.k)
    st, rhs = boxmg.discretize(kk, dev(p.f))
    H = ref.Hierarchy(host(st))
    return p, kk, st, rhs, H


def test_fused_passes_4095(gpu, jumping4095):
    """The pre pass (two sweeps, residual, restriction; weights computed in the
    pass on the five-point level) and the post pass (interpolation, one sweep)
    on levels 0 (4095^2) and 1 (2047^2), as the solve launches them."""
    p, kk, st, rhs, H = jumping4095
    S = boxmg.Solver(st)
    rng = np.random.default_rng(4095)
    for l in (0, 1):
        nl, nc = H.level_n(l), H.level_n(l + 1)
        op, Ci = H.op(l), H.field(l, "Ci")
        u, b = rand_level(rng, nl), rand_level(rng, nl)
        S.import_(l, "u", dev(u)); S.import_(l, "b", dev(b))
        S.import_(l + 1, "u", dev(rand_level(rng, nc)))
        S.step(l, "pre", 2)
        us = ref.gs(*op, b, u, 2)
        same(host(S.export(l, "u")), us, f"pre u l={l}")
        same(host(S.export(l + 1, "b")), ref.restrict(Ci, ref.residual(*op, b, us)), f"pre b_c l={l}")
        assert not host(S.export(l + 1, "u")).any()
        ec = rand_level(rng, nc)
        S.import_(l, "u", dev(u)); S.import_(l, "b", dev(b)); S.import_(l + 1, "u", dev(ec))
        S.step(l, "post", 1)
        same(host(S.export(l, "u")), ref.gs(*op, b, ref.interp_add(Ci, ec, u), 1), f"post u l={l}")
    S.close()


def test_first_cycles_4095(gpu, jumping4095):
    """Three cycles of the benchmark's solve (every level, the small-level
    kernel, the fine post pass run with the next cycle's fine pre pass and
    the norm inside it, in the benchmark's launch configuration) equal the
    oracle's."""
    p, kk, st, rhs, H = jumping4095
    S = boxmg.Solver(st, max_cycles=3, check_every=16)
    x, info = S.solve(rhs, tol=1e-10, raise_on_noconv=False)
    u, hist = H.solve(ref.pad(host(rhs)), tol=1e-10, max_cycles=3)
    assert info["cycles"] == len(hist) == 3
    same(host(x), u[1:-1, 1:-1], "iterate after 3 cycles")
    assert np.all(np.abs(np.array(info["history"]) - hist) <= 1e-12 * hist)
    S.close()


def test_block_first_cycles_4095(gpu, jumping4095):
    """Two cycles of a two-right-hand-side block on the benchmark's operator,
    each right-hand side against the oracle."""
    p, kk, st, rhs, H = jumping4095
    n = p.n
    rhs2 = torch.stack([boxmg.discretize(kk, dev(f))[1] for f in inputs.extra_sources(n, 2)])
    S = boxmg.Solver(st, max_cycles=2, check_every=16)
    B = boxmg.Block(S, 2)
    xb, infos = B.solve(rhs2, tol=1e-10, raise_on_noconv=False)
    for j in range(2):
        u, hist = H.solve(ref.pad(host(rhs2[j])), tol=1e-10, max_cycles=2)
        assert infos[j]["cycles"] == len(hist) == 2
        same(host(xb[j]), u[1:-1, 1:-1], f"rhs {j}")
    B.close()
    S.close()


def test_fp32_pre_pass_8191(gpu):
    """The FP32 hierarchy's fine pre pass at 8191^2 (the FP32-refinement
    workload) against the oracle's FP32 steps."""
    p = inputs.jumping_8191()
    st, _ = boxmg.discretize(dev(p.k), dev(p.f))
    S = boxmg.Solver(st, precision=boxmg.BMG_FP32_IR)
    H = ref.Hierarchy(host(st))
    f32 = np.float32
    op = tuple(None if a is None else a.astype(f32) for a in H.op(0))
    Ci = H.field(0, "Ci").astype(f32)
    rng = np.random.default_rng(8191)
    n0, n1 = H.level_n(0), H.level_n(1)
    u, b = rand_level(rng, n0, f32), rand_level(rng, n0, f32)
    S.import_(0, "u32", dev(u)); S.import_(0, "b32", dev(b))
    S.import_(1, "u32", dev(rand_level(rng, n1, f32)))
    S.step(0, "pre", 2, fp32=True)
    us = ref.gs(*op, b, u, 2, dtype=f32)
    same(host(S.export(0, "u32")), us, "pre u")
    same(host(S.export(1, "b32")), ref.restrict(Ci, ref.residual(*op, b, us, dtype=f32), dtype=f32), "pre b_c")
    S.close()
