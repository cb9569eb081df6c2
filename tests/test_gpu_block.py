"""Block solves (several right-hand sides on one hierarchy) against the single
solve and the oracle.  Each right-hand side must follow its own solve exactly:
the same cycle count, the same switch to double-FP64 refinement, the same
iterate bit for bit, whatever the other right-hand sides in the block do."""
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


def block_problem(n, k, seed, zero=()):
    """One jumping-coefficient operator and k right-hand sides h^2 f_j."""
    p = inputs.jumping(n, 16 if n >= 31 else 2, -2, 2, 300 + seed, 400 + seed)
    kk = dev(p.k)
    st, _ = boxmg.discretize(kk, dev(p.f))
    rhs = []
    for j in range(k):
        f = np.zeros((n, n)) if j in zero else inputs.uniform_source(n, 1000 * seed + j)
        rhs.append(boxmg.discretize(kk, dev(f))[1])
    return st, torch.stack(rhs)


@pytest.mark.parametrize("n,k,tile_rows", [(255, 5, 0), (127, 3, 6), (7, 2, 0)])
def test_block_equals_single_solves(gpu, n, k, tile_rows):
    """Every right-hand side of a block (one of them zero, one with a nonzero
    initial guess) equals its own bmg_solve: cycles and both parts of the
    iterate bit for bit, history to 1e-12 (the norm's per-tile partial sums
    follow the tiling of the pass that takes it: the block's post pass, or the
    single solve's fused post and next pre pass)."""
    st, rhs = block_problem(n, k, 7, zero=(1,))
    x0 = torch.zeros_like(rhs)
    x0[k - 1] = dev(np.random.default_rng(5).uniform(-1e-3, 1e-3, size=(n, n)))
    S = boxmg.Solver(st, max_cycles=400, tile_rows=tile_rows)
    B = boxmg.Block(S, k)
    xb, infos = B.solve(rhs, x0.clone(), tol=1e-10, raise_on_noconv=False)
    for j in range(k):
        x1, i1 = S.solve(rhs[j].contiguous(), x0[j].clone(), tol=1e-10, raise_on_noconv=False)
        assert infos[j]["cycles"] == i1["cycles"], (j, infos[j]["cycles"], i1["cycles"])
        h, h1 = np.array(infos[j]["history"]), np.array(i1["history"])
        assert np.all(np.abs(h - h1) <= 1e-12 * h1), j
        assert infos[j]["status"] == i1["status"], j
        same(host(xb[j]), host(x1), f"rhs {j}")
    assert all(i["status"] == 0 for i in infos), [i["rel_res"] for i in infos]
    assert infos[1]["cycles"] == 0 and not host(xb[1]).any()
    counts = [i["cycles"] for j, i in enumerate(infos) if j != 1]
    if n >= 255:
        assert len(set(counts)) > 1   # the right-hand sides stop at different cycles
    B.close()
    S.close()


def test_block_matches_oracle(gpu):
    """Each right-hand side of a block against the oracle's solve (several
    strips and row tiles, refinement below the FP64 floor)."""
    n, k = 255, 3
    st, rhs = block_problem(n, k, 11)
    S = boxmg.Solver(st, max_cycles=300)
    B = boxmg.Block(S, k)
    xb, infos = B.solve(rhs, tol=1e-10, raise_on_noconv=False)
    H = ref.Hierarchy(host(st))
    for j in range(k):
        u, hist = H.solve(ref.pad(host(rhs[j])), tol=1e-10, max_cycles=300)
        assert infos[j]["cycles"] == len(hist)
        same(host(xb[j]), u[1:-1, 1:-1], f"rhs {j}")
        h = np.array(infos[j]["history"])
        assert np.all(np.abs(h - hist) <= 1e-12 * hist)


def test_block_max_cycles(gpu):
    """A block stopped by max_cycles reports ENOCONV for each right-hand side,
    with the iterates of single solves stopped the same way."""
    n, k = 127, 3
    st, rhs = block_problem(n, k, 3)
    S = boxmg.Solver(st, max_cycles=5)
    B = boxmg.Block(S, k)
    xb, infos = B.solve(rhs, tol=1e-10, raise_on_noconv=False)
    for j in range(k):
        x1, i1 = S.solve(rhs[j].contiguous(), tol=1e-10, raise_on_noconv=False)
        assert infos[j]["status"] == boxmg.BMG_ENOCONV == i1["status"]
        assert infos[j]["cycles"] == 5 == i1["cycles"]
        same(host(xb[j]), host(x1), f"rhs {j}")
    with pytest.raises(boxmg.BoxMGError) as e:
        B.solve(rhs, tol=1e-10)
    assert e.value.status == boxmg.BMG_ENOCONV


def test_block_trace_counts_shared_bytes(gpu):
    """The operator and the weights count once per launch, the iterates and
    right-hand sides k times (the five-point pre pass reads its weights when
    it runs several right-hand sides)."""
    n, k = 255, 4
    st, rhs = block_problem(n, k, 5)
    S = boxmg.Solver(st, max_cycles=3)
    B = boxmg.Block(S, k)
    n0, n1 = S.level_n(0), S.level_n(1)
    B.trace_enable("pre", 0)
    B.solve(rhs, tol=1e-10, raise_on_noconv=False)
    nl, ms, nb = B.trace_read()
    assert nl >= 3 and ms > 0
    assert nb == nl * 8 * ((3 + 3 * k) * n0 * n0 + (2 * k + 8) * n1 * n1)
    B.trace_enable("post", 1)
    B.solve(rhs, tol=1e-10, raise_on_noconv=False)
    nl, ms, nb = B.trace_read()
    n2 = S.level_n(2)
    assert nl >= 3 and nb == nl * 8 * ((5 + 3 * k) * n1 * n1 + (k + 8) * n2 * n2)


def test_block_rejects_what_it_cannot_run(gpu):
    st, rhs = block_problem(127, 2, 1)
    for opts in (dict(precision=boxmg.BMG_FP32_IR), dict(kernels=boxmg.BMG_KERNELS_BASIC), dict(nu1=4)):
        S = boxmg.Solver(st, **opts)
        with pytest.raises(boxmg.BoxMGError) as e:
            boxmg.Block(S, 2)
        assert e.value.status == boxmg.BMG_EINVAL
    S = boxmg.Solver(st)
    with pytest.raises(boxmg.BoxMGError):
        boxmg.Block(S, 0)
