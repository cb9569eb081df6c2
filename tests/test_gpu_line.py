"""Line relaxation on the GPU against the oracle, element by element: the
relaxation steps of five- and nine-point levels (several transpose tiles and
a ragged last one), and whole solves with the line smoother."""
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


def rand_level(rng, n):
    a = np.zeros((n + 2, n + 2))
    a[1:-1, 1:-1] = rng.standard_normal((n, n))
    return a


def anisotropic_jumping(n, seed, ax=100.0):
    """The oracle's jumping-coefficient operator with its interior x-couplings
    scaled by ax and the centre raised by the same amount, so the rows keep
    their sums (a symmetric M-matrix that couples strongly along x)."""
    p = inputs.jumping(n, 16 if n >= 31 else 2, -2, 2, seed, seed + 1)
    st, rhs = ref.discretize(p.k, p.f)
    st = st.copy()
    w, e = st[:, :, 1].copy(), st[:, :, 3].copy()
    st[:, :, 1] *= ax
    st[:, :, 3] *= ax
    st[:, :, 2] = st[:, :, 2] - (ax - 1.0) * (w + e)
    return st, rhs


@pytest.mark.parametrize("n", [7, 127, 255])
def test_line_relaxation_steps_bitwise(gpu, n):
    """Two relaxations on every level of the hierarchy equal the oracle's."""
    p = inputs.jumping(n, 16 if n >= 31 else 2, -3, 3, 21, 22)
    st, _ = boxmg.discretize(dev(p.k), dev(p.f))
    S = boxmg.Solver(st, smoother=boxmg.BMG_SMOOTH_LINE)
    H = ref.Hierarchy(host(st))
    rng = np.random.default_rng(n)
    for l in range(H.nlev):
        nl = H.level_n(l)
        op = H.op(l)
        u, b = rand_level(rng, nl), rand_level(rng, nl)
        S.import_(l, "u", dev(u)); S.import_(l, "b", dev(b))
        S.step(l, "smooth", 2)
        want = ref.line_relax(*op, ref.line_factor(*op[:3]), b, u, 2)
        same(host(S.export(l, "u")), want, f"level {l} (n={nl})")
    S.close()


@pytest.mark.parametrize("n,ax", [(255, 1.0), (127, 100.0)])
def test_line_solve_matches_oracle(gpu, n, ax):
    """Solves with the line smoother: cycles, iterate (both parts) bitwise,
    history to 1e-12, on an isotropic and an anisotropic operator."""
    st_h, rhs_h = anisotropic_jumping(n, 31, ax)
    st, rhs = dev(st_h), dev(rhs_h)
    S = boxmg.Solver(st, smoother=boxmg.BMG_SMOOTH_LINE, max_cycles=200)
    x, info = S.solve(rhs, tol=1e-10, raise_on_noconv=False)
    H = ref.Hierarchy(st_h, smoother="line")
    u, hist = H.solve(ref.pad(rhs_h), tol=1e-10, max_cycles=200)
    assert info["cycles"] == len(hist) and info["status"] == 0
    same(host(x), u[1:-1, 1:-1], "solution (high part)")
    same(host(S.export(0, "xlo")), H.xl, "solution (low part)")
    h = np.array(info["history"])
    assert np.all(np.abs(h - hist) <= 1e-12 * hist)
    S.close()


def test_line_smoother_restrictions(gpu):
    p = inputs.jumping(63, 16, -2, 2, 1, 2)
    st, _ = boxmg.discretize(dev(p.k), dev(p.f))
    with pytest.raises(boxmg.BoxMGError) as e:
        boxmg.Solver(st, smoother=boxmg.BMG_SMOOTH_LINE, precision=boxmg.BMG_FP32_IR)
    assert e.value.status == boxmg.BMG_EINVAL
    S = boxmg.Solver(st, smoother=boxmg.BMG_SMOOTH_LINE)
    with pytest.raises(boxmg.BoxMGError):
        S.step(0, "pre", 2)
    with pytest.raises(boxmg.BoxMGError):
        boxmg.Block(S, 2)
