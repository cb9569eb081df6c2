"""Parity at the workloads' full sizes, in the launch configuration bench.py
times: default options, hence the default tile heights of the large levels
and the weights computed in the fine pre pass.  Whole levels are compared
element by element; the oracle's C tier finishes a 4095^2 set-up in seconds.
The inputs are the benchmark's own (the 4095^2 jumping-coefficient field and
its source, and for the FP32 refinement the 8191^2 field); the whole solves use
the benchmark's coarsest level (63^2 on these fields), so every kernel a timed
solve launches, refinement steps included, is compared at the timed size."""
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


HEADLINE_COARSEST = 63   # the directly solved level of the jumping-coefficient workloads


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


def test_headline_solve_4095(gpu, jumping4095):
    """The benchmark's whole solve (4095^2, coarsest 63^2, default tiles): the
    plain FP64 cycles, the switch at 16 tol and the double-FP64 refinement
    steps (fine post pass with the iterate update, accurate outer residual)
    to 1e-10.  Cycle count, both parts of the iterate bit for bit, history to
    1e-12."""
    p, kk, st, rhs, _ = jumping4095
    H = ref.Hierarchy(host(st), coarsest=HEADLINE_COARSEST)
    u, hist = H.solve(ref.pad(host(rhs)), tol=1e-10, max_cycles=200)
    with boxmg.Solver(st, max_cycles=200, coarsest_n=HEADLINE_COARSEST) as S:
        x, info = S.solve(rhs, tol=1e-10)
        assert info["cycles"] == len(hist), (info["cycles"], len(hist))
        assert hist[-2] > 1e-10 >= hist[-1]
        assert (hist > 16e-10).sum() < len(hist) - 1      # some refinement steps ran
        same(host(x), u[1:-1, 1:-1], "solution (high part)")
        same(host(S.export(0, "xlo")), H.xl, "solution (low part)")
        h = np.array(info["history"])
        assert np.all(np.abs(h - hist) <= 1e-12 * hist), np.abs(h / hist - 1).max()
    H.close()


def test_line_relaxation_every_level_4095(gpu, jumping4095):
    """One alternating zebra line relaxation on every level of the benchmark's
    line-smoother hierarchy (4095^2 down to 63^2), as bench.py --smoother line
    launches it."""
    p, kk, st, rhs, _ = jumping4095
    H = ref.Hierarchy(host(st), coarsest=HEADLINE_COARSEST)
    rng = np.random.default_rng(40951)
    with boxmg.Solver(st, smoother=boxmg.BMG_SMOOTH_LINE, coarsest_n=HEADLINE_COARSEST) as S:
        assert S.nlev == H.nlev
        for l in range(H.nlev - 1):
            nl = H.level_n(l)
            op = H.op(l)
            u, b = rand_level(rng, nl), rand_level(rng, nl)
            S.import_(l, "u", dev(u)); S.import_(l, "b", dev(b))
            S.step(l, "smooth", 1)
            want = ref.line_relax(*op, ref.line_factor(*op[:3]), b, u, 1)
            same(host(S.export(l, "u")), want, f"level {l} (n={nl})")
    H.close()


@pytest.fixture(scope="module")
def jumping8191():
    p = inputs.jumping_8191()
    st, rhs = boxmg.discretize(dev(p.k), dev(p.f))
    return p, st, rhs


def test_fp32_refinement_solve_8191(gpu, jumping8191):
    """The FP32-refinement workload's whole solve at 8191^2 (coarsest 63^2):
    every step (FP64 outer residual with the max-norm scaling, FP32 V-cycle
    with its fine pre pass reading the residual and its fine post pass
    updating the double-FP64 iterate) equals the oracle's bit for bit.  The
    refined solution is then compared with the oracle's plain FP64 solve of
    the same problem: the error of the mixed-precision form against the FP64
    oracle, printed and bounded."""
    p, st, rhs = jumping8191
    H = ref.Hierarchy(host(st), coarsest=HEADLINE_COARSEST)
    b = ref.pad(host(rhs))
    u, hist = H.solve_ir(b, tol=1e-10, max_iter=200)
    ul = H.xl.copy()
    with boxmg.Solver(st, max_cycles=200, coarsest_n=HEADLINE_COARSEST, precision=boxmg.BMG_FP32_IR) as S:
        x, info = S.solve(rhs, tol=1e-10)
        assert info["cycles"] == len(hist) - 1, (info["cycles"], len(hist) - 1)
        same(host(x), u[1:-1, 1:-1], "refined solution (high part)")
        same(host(S.export(0, "xlo")), ul, "refined solution (low part)")
    v, hist64 = H.solve(b, tol=1e-10, max_cycles=200)
    d = (u - v) + (ul - H.xl)
    err2 = np.linalg.norm(d) / np.linalg.norm(v + H.xl)
    errinf = np.abs(d).max() / np.abs(v + H.xl).max()
    print(f"8191^2: FP32-in-refinement {len(hist) - 1} steps, FP64 {len(hist64)} cycles; "
          f"solution error against the FP64 oracle: {err2:.3e} (2-norm), {errinf:.3e} (max-norm)")
    # both residuals are <= 1e-10 relative; ||A^-1|| ||b|| / ||x|| bounds the
    # error's amplification, about 1e3 on these fields
    assert err2 < 1e-9 and errinf < 1e-9
    H.close()


def test_batch_with_1023_problems(gpu):
    """A batch that holds every size of the batched workload, 1023^2 included,
    solved with the tile height the benchmark's tuner picks (32 rows on every
    level): each problem's solution and step count equal the oracle's
    FP32-in-double-FP64 refinement bit for bit."""
    probs = inputs.batch_512(count=10, m_lo=6, m_hi=10, seed=404)
    assert {q.n for q in probs} == {63, 127, 255, 511, 1023}, sorted(q.n for q in probs)
    old = {n: boxmg.tile_rows_get(n) for n in (63, 127, 255, 511, 1023)}
    try:
        for n in old:
            boxmg.tile_rows_set(n, 32)
        sts, rhss = [], []
        for q in probs:
            st, rhs = boxmg.discretize(dev(q.k), dev(q.f))
            sts.append(st)
            rhss.append(rhs)
        with boxmg.Batch(sts, max_cycles=80) as B:
            x, steps, rel, status = B.solve(rhss, tol=1e-10)
            assert status == boxmg.BMG_OK
            for p, q in enumerate(probs):
                H = ref.Hierarchy(host(sts[p]))
                u, hist = H.solve_ir(ref.pad(host(rhss[p])), tol=1e-10, max_iter=80)
                assert steps[p] == len(hist) - 1, (p, q.n)
                same(host(x[p]), u[1:-1, 1:-1], f"problem {p} (n={q.n})")
                H.close()
    finally:
        for n, r in old.items():
            boxmg.tile_rows_set(n, r)
