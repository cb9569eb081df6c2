"""Nonsymmetric BoxMG on the GPU against the CPU oracle, element by element:
the set-up (full stencils of every level, the weights of P and R, the
coarsest L D U factor), every step of the cycle on every level, and whole
solves, on convection-diffusion operators (diffusion stencil plus the upwind
convection part of the input generator)."""
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


def cd_problem(n, beta, flow="rotating", block=None, lo=-1.0, hi=1.0, seed=5, nine=False):
    """A convection-diffusion stencil (five-point, or as nine entries per row
    with zero corners) and its right-hand side, from the oracle's
    discretisation (bitwise the GPU's) plus the upwind convection input."""
    p = inputs.jumping(n, block or max(2, (n + 1) // 8), lo, hi, seed, seed + 1)
    st, rhs = ref.discretize(p.k, p.f)
    st = st + inputs.upwind_convection(n, beta, flow)
    if nine:
        full = np.zeros((n, n, 9))
        full[:, :, [1, 3, 4, 5, 7]] = st
        st = full
    return st, rhs


CASES = [(31, 20.0, 3, False), (127, 60.0, 15, False), (255, 40.0, 31, True), (255, 80.0, 63, False)]


@pytest.mark.parametrize("n,beta,nc,nine", CASES)
def test_ns_setup_bitwise(gpu, n, beta, nc, nine):
    st, _ = cd_problem(n, beta, nine=nine)
    H = ref.NSHierarchy(st, coarsest=nc)
    with boxmg.NSSolver(dev(st), coarsest_n=nc) as S:
        assert S.nlev == H.nlev
        for l in range(H.nlev):
            for e in range(9):
                same(host(S.export(l, f"A{e}")), H.field(l, f"A{e}"), f"level {l} plane {e}")
            if l + 1 < H.nlev:
                same(host(S.export(l, "Pi")), H.field(l, "Pi"), f"level {l} P")
                same(host(S.export(l, "Ri")), H.field(l, "Ri"), f"level {l} R")
        Lb, Ub, D = H.coarse_factor()
        f = host(S.export(0, "LDU"))
        m, w = Lb.shape
        same(f[:m * w].reshape(m, w), Lb, "L")
        same(f[m * w:2 * m * w].reshape(m, w), Ub, "U")
        same(f[2 * m * w:], D, "D")


@pytest.mark.parametrize("n,beta,nc,nine", CASES[:3])
def test_ns_steps_bitwise(gpu, n, beta, nc, nine):
    """Two sweeps, the residual, the restriction with R, the interpolation with
    P on every level, and the coarsest solve, each from the same random
    arrays on both sides."""
    st, _ = cd_problem(n, beta, nine=nine)
    H = ref.NSHierarchy(st, coarsest=nc)
    rng = np.random.default_rng(n)
    with boxmg.NSSolver(dev(st), coarsest_n=nc) as S:
        for l in range(H.nlev):
            nl = H.level_n(l)
            u, b = ref.pad(rng.standard_normal((nl, nl))), ref.pad(rng.standard_normal((nl, nl)))
            H.set_field(l, "u", u)
            H.set_field(l, "b", b)
            S.import_(l, "u", dev(u))
            S.import_(l, "b", dev(b))
            if l == H.nlev - 1:
                H.step(l, "coarse")
                S.step(l, "coarse")
                same(host(S.export(l, "u")), H.field(l, "u"), f"coarsest solve (n={nl})")
                continue
            H.step(l, "smooth", 2)
            S.step(l, "smooth", 2)
            same(host(S.export(l, "u")), H.field(l, "u"), f"level {l} sweeps")
            H.step(l, "residual")
            S.step(l, "residual")
            same(host(S.export(l, "r")), H.field(l, "r"), f"level {l} residual")
            H.step(l, "restrict")
            S.step(l, "restrict")
            same(host(S.export(l + 1, "b")), H.field(l + 1, "b"), f"level {l} restriction")
            ec = ref.pad(rng.standard_normal((H.level_n(l + 1), H.level_n(l + 1))))
            H.set_field(l + 1, "u", ec)
            S.import_(l + 1, "u", dev(ec))
            H.step(l, "interp")
            S.step(l, "interp")
            same(host(S.export(l, "u")), H.field(l, "u"), f"level {l} interpolation")


@pytest.mark.parametrize("n,beta,flow,nc", [(127, 30.0, "rotating", 3), (255, 80.0, "constant", 15),
                                             (511, 60.0, "rotating", 63), (1023, 100.0, "rotating", 63)])
def test_ns_solve_matches_oracle(gpu, n, beta, flow, nc):
    """Whole solves to 1e-10: cycle count and the iterate bit for bit, the
    residual history to 1e-12 (the norms' sums run in another order)."""
    st, rhs = cd_problem(n, beta, flow, block=16)
    H = ref.NSHierarchy(st, coarsest=nc)
    u, hist = H.solve(ref.pad(rhs), tol=1e-10, max_cycles=100)
    with boxmg.NSSolver(dev(st), coarsest_n=nc, max_cycles=100) as S:
        x, info = S.solve(dev(rhs), tol=1e-10)
        assert info["cycles"] == len(hist)
        same(host(x), u[1:-1, 1:-1], "solution")
        h = np.array(info["history"])
        assert np.all(np.abs(h - hist) <= 1e-12 * hist), np.abs(h / hist - 1).max()


def test_ns_rejects_and_reports(gpu):
    st, rhs = cd_problem(31, 10.0)
    bad = st.copy()
    bad[0, 5, 0] = -1.0                          # coupling to the boundary
    with pytest.raises(boxmg.BoxMGError) as e:
        boxmg.NSSolver(dev(bad))
    assert e.value.status == boxmg.BMG_EINVAL
    with pytest.raises(boxmg.BoxMGError):
        boxmg.NSSolver(dev(st), precision=boxmg.BMG_FP32_IR)
    with boxmg.NSSolver(dev(st), max_cycles=2) as S:
        x, info = S.solve(dev(rhs), tol=1e-14, raise_on_noconv=False)
        assert info["status"] == boxmg.BMG_ENOCONV and info["cycles"] == 2
        x, info = S.solve(torch.zeros_like(dev(rhs)), tol=1e-10)
        assert info["cycles"] == 0 and not x.any()
