"""Benchmark: fine-grid DOF/s of a BoxMG solve to a 1e-10 relative residual.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload jumping_4095]

One step = the whole hot path on one synthetic problem already resident in HBM:
set-up (interpolation weights, Galerkin coarse operators, coarsest factor) and
the V(2,1) solve to the tolerance.  The discretisation of the seeded
coefficients is done once, before timing (it is the problem's input).

Printed: one JSON line with the throughput, the dominant kernel's achieved
HBM bandwidth against the MI355X peak (HIP events around its launches on the
solver's stream, inside the timed region) and the CPU oracle timed on this
host on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fine DOF/s solved to 1e-10 rel. residual (4095^2); smoother HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0

# The algorithmic bytes of the timed launches come from the library, which
# counts each array a launch needs once (read or written) for the variant that
# ran: a five-point FP64 pre pass reads A_O, A_W, A_S, b, u and writes u (48 B
# per fine point) and writes b_c, u_c (16 B per coarse point: 4 per fine point),
# 52 B per fine point, as it computes the interpolation weights itself; with
# stored weights their 8 planes add 16 B per fine point.


KERNEL_NAMES = {"postpre": "k_postpre (fine post pass with the next cycle's fine pre pass)",
                "pre": "k_pre (fine pre pass)", "resnorm": "k_resid_dd (FP64 outer residual)",
                "smooth": "k_gs_colour / line relaxation (fine level)"}


def measured_traffic(key: str, tile_rows: int | None = None):
    """HBM bytes per launch of the timed kernel from the committed counter
    record (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a copy
    of known size), or None when there is none for this run, or the kernel's
    sources or its launch geometry (rows per tile) have changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None
    if not rec:
        return None
    if tile_rows is not None and rec.get("tile_rows") not in (None, tile_rows):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        try:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        except OSError:
            return None
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def workload(name: str):
    from paper_2502_05279_amd import inputs
    if name == "jumping_4095":
        return inputs.jumping_4095()
    if name == "poisson_127":
        return inputs.poisson_127()
    if name == "jumping_8191":
        return inputs.jumping_8191()
    if name.startswith("jumping_"):
        n = int(name.split("_")[1])
        return inputs.jumping_4095(n=n)
    raise SystemExit(f"unknown workload {name}")


def default_coarsest(name: str, n: int) -> int:
    """Points per side of the directly solved coarsest level.  The 127^2
    Poisson workload fixes 3x3.  On the block-wise jumping fields the coarsest
    level is the last one whose grid lines still carry every coefficient jump
    (64-cell blocks at 4095^2, 128-cell blocks at 8191^2: the 63^2 level), the
    largest the one-wave band solve takes."""
    if name.startswith("jumping_") or name.startswith("learned"):
        return min(63, n)
    return 3


def omp_threads() -> int:
    try:
        import ctypes
        return ctypes.CDLL("libgomp.so.1").omp_get_max_threads()
    except OSError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_solve_times(p, coarsest: int, tol: float, threads: int | None = None):
    """The oracle's whole solve on this host: (set-up s, solve s, cycles).
    threads: OpenMP threads (None = all), with the process pinned to that many
    cores while it runs."""
    import ctypes
    from oracle import ref
    gomp = ctypes.CDLL("libgomp.so.1")
    st, rhs = ref.discretize(p.k, p.f)
    b = ref.pad(rhs)
    old_aff = os.sched_getaffinity(0)
    old_thr = gomp.omp_get_max_threads()
    try:
        if threads:
            os.sched_setaffinity(0, set(sorted(old_aff)[:threads]))
            gomp.omp_set_num_threads(threads)
        t0 = time.perf_counter()
        H = ref.Hierarchy(st, coarsest=coarsest)
        t1 = time.perf_counter()
        u, hist = H.solve(b, tol=tol, max_cycles=2000)
        t2 = time.perf_counter()
        H.close()
        print(f"cpu baseline: oracle solve on {threads or 'all'} thread(s): set-up {t1 - t0:.2f} s, "
              f"{len(hist)} cycles {t2 - t1:.2f} s", file=sys.stderr, flush=True)
    finally:
        gomp.omp_set_num_threads(old_thr)
        os.sched_setaffinity(0, old_aff)
    return t1 - t0, t2 - t1, len(hist)


def cpu_baseline(p, coarsest: int, tol: float, full: bool):
    """The oracle solving the same problem on this host's cores: set-up and the
    solve to the tolerance timed separately, no extrapolation.  Default: one
    solve on all cores.  full: the median of 3 on all cores and of 3 on one
    core."""
    runs = 3 if full else 1
    allc = [oracle_solve_times(p, coarsest, tol) for _ in range(runs)]
    med = sorted(allc, key=lambda r: r[0] + r[1])[len(allc) // 2]
    out = {"value": p.n * p.n / (med[0] + med[1]), "unit": "DOF/s", "cores": omp_threads(),
           "kind": "oracle", "cpu": cpu_model(),
           "setup_s": med[0], "solve_s": med[1], "cycles": med[2],
           "sample": f"the whole {p.n}^2 solve to {tol:g} (set-up + {med[2]} cycles, coarsest "
                     f"{coarsest}^2), {'median of 3' if full else 'one run'} on all host cores"}
    if full:
        one = [oracle_solve_times(p, coarsest, tol, threads=1) for _ in range(runs)]
        m1 = sorted(one, key=lambda r: r[0] + r[1])[len(one) // 2]
        out["one_core"] = {"value": p.n * p.n / (m1[0] + m1[1]), "setup_s": m1[0], "solve_s": m1[1],
                           "cycles": m1[2], "runs": runs}
    return out


def bench_batch(args):
    """512 independent problems of uneven size (2^m - 1, m in 6..10, per-cell
    log-normal k), solved together: FP32 V-cycles inside double-FP64 refinement
    in one persistent launch per group of steps, tile heights from the
    autotuner.  One step = set-up of all problems + the batched solve."""
    import torch
    from paper_2502_05279_amd import autotune, boxmg, inputs

    dev = torch.device("cuda:0")
    sizes = (63, 127, 255, 511, 1023)
    probs = inputs.batch_512()
    sts, rhss = [], []
    for q in probs:
        st, rhs = boxmg.discretize(torch.from_numpy(q.k).to(dev), torch.from_numpy(q.f).to(dev))
        sts.append(st)
        rhss.append(rhs)
    dof = sum(q.n * q.n for q in probs)

    def step():
        B = boxmg.Batch(sts, max_cycles=args.max_cycles)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, steps, rel, status = B.solve(rhss, tol=args.tol, raise_on_noconv=False)
        torch.cuda.synchronize()
        return B, x, steps, rel, status, time.perf_counter() - t1

    if args.batch_tile_rows:
        tuned = {n: args.batch_tile_rows for n in sizes}
        for n, r in tuned.items():
            boxmg.tile_rows_set(n, r)
    else:
        # untimed: one batched solve per candidate tile height
        def tune_once():
            out = step()
            out[0].close()
            return out[-1]
        tuned = autotune.tune_batch(tune_once, sizes)
    for _ in range(args.warmup):
        step()[0].close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solve_s = 0.0
    for k in range(args.steps):
        B, x, steps, rel, status, ts = step()
        solve_s += ts
        if k + 1 < args.steps:
            B.close()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    info = B.info()
    B.close()
    sizes = sorted({q.n for q in probs})
    out = {
        "metric": f"fine DOF/s solved to {args.tol:g} rel. residual (512 problems, FP32 V-cycle in FP64 refinement)",
        "value": dof / dt, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batch_512", "problems": len(probs), "dof": dof,
                   "sizes": {str(n): sum(q.n == n for q in probs) for n in sizes},
                   "tol": args.tol, "solve_ms": solve_s / args.steps * 1e3,
                   "solve_dof_per_s": dof / (solve_s / args.steps),
                   "steps_max": max(steps), "steps_mean": sum(steps) / len(steps),
                   "max_rel_res": max(rel), "converged": status == 0,
                   "workgroups": info["workgroups"], "graph": info["graph"],
                   "tile_rows": {str(k): v for k, v in tuned.items()},
                   "tile_ms": {str(k): {str(r): round(t, 4) for r, t in v.items()}
                               for k, v in autotune.LAST.items()}},
    }
    print(json.dumps(out))


def bench_learned(args):
    """Learned interpolation against BoxMG's on a 4095^2 field of contrast 1e6:
    one step = BoxMG set-up, learned set-up (network on every level), two
    probe cycles on each hierarchy and the solve to the tolerance with the one
    whose probe factor is smaller.  BoxMG alone and the learned hierarchy
    alone are timed beside it (reported in config)."""
    import torch
    from paper_2502_05279_amd import boxmg, inputs, learned

    dev = torch.device("cuda:0")
    params = learned.load_params(args.params or learned.DEFAULT_PARAMS)
    p = inputs.learned_eval_4095(n=args.learned_n)
    n = p.n
    st, rhs = boxmg.discretize(torch.from_numpy(p.k).to(dev), torch.from_numpy(p.f).to(dev))
    net = boxmg.Net(params, max_n=n, train=False)
    opts = dict(max_cycles=args.max_cycles, check_every=16,
                coarsest_n=args.coarsest or default_coarsest("learned", n))

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def run_boxmg():
        with boxmg.Solver(st, **opts) as B:
            return B.solve(rhs, tol=args.tol, raise_on_noconv=False)

    # a learned set-up can break down (a coarse operator built with learned
    # weights on which BoxMG's formula has a denominator <= 0): the step then
    # solves with BoxMG alone, the fallback, and the line says so
    broke = []

    def run_learned():
        try:
            with boxmg.Solver(st, interp=boxmg.BMG_INTERP_LEARNED, net=net, **opts) as L:
                return L.solve(rhs, tol=args.tol, raise_on_noconv=False)
        except boxmg.BoxMGError as e:
            if e.status != boxmg.BMG_EBREAKDOWN:
                raise
            broke.append(str(e))
            return None, None

    def run_select():
        try:
            L = boxmg.Solver(st, interp=boxmg.BMG_INTERP_LEARNED, net=net, **opts)
        except boxmg.BoxMGError as e:
            if e.status != boxmg.BMG_EBREAKDOWN:
                raise
            broke.append(str(e))
            x, info = run_boxmg()
            return x, info, boxmg.BMG_INTERP_BOXMG, (None, None)
        with L, boxmg.Solver(st, **opts) as B:
            return boxmg.solve_select(L, B, rhs, tol=args.tol, raise_on_noconv=False)

    for _ in range(args.warmup):
        run_select()
    (_, ib), tb = timed(run_boxmg)
    (_, il), tl = timed(run_learned)
    il = il or {"cycles": None, "rho": None, "rel_res": None}
    times = []
    for _ in range(args.steps):
        (x, info, used, rho), ts = timed(run_select)
        times.append(ts)
    dt = float(np.mean(times))
    out = {
        "metric": f"fine DOF/s solved to {args.tol:g} rel. residual ({n}^2, contrast 1e6), learned "
                  "interpolation with BoxMG fallback",
        "value": n * n / dt, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (network bf16/f32)", "data": "synthetic",
        "config": {"workload": f"learned_eval_{n}", "n": n, "tol": args.tol,
                   "used": "learned" if used == boxmg.BMG_INTERP_LEARNED else "boxmg",
                   "probe_rho_learned": rho[0], "probe_rho_boxmg": rho[1],
                   "cycles": info["cycles"], "final_rel_res": info["rel_res"],
                   "boxmg_ms": tb * 1e3, "boxmg_cycles": ib["cycles"], "boxmg_rho": ib["rho"],
                   "learned_ms": tl * 1e3, "learned_cycles": il["cycles"], "learned_rho": il["rho"],
                   "learned_final_rel_res": il["rel_res"],
                   "learned_setup": broke[0] if broke else "ok"},
    }
    # the network's forward pass on the fine operator, the learned set-up's
    # dominant work: conv1 (9 -> 32 channels, 3x3) at every fine point, conv2
    # (32 -> 32, stride 2) and conv3 (32 -> 8) at the (nc+1)^2 coarse points,
    # 2 flop per multiply-add, on bfloat16 MFMA
    S0 = boxmg.Solver(st, **opts)
    planes = [S0.export(0, f) for f in ("O", "W", "S")]
    nc = (n - 1) // 2
    Ci = torch.zeros((8, nc + 2, nc + 2), dtype=torch.float64, device=dev)
    net.forward(*planes, out=Ci)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        net.forward(*planes, out=Ci)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    flop = 2.0 * (9 * 9 * 32) * n * n + 2.0 * (32 * 9 * 32 + 32 * 9 * 8) * (nc + 1) ** 2
    tflops = flop / (fwd_ms * 1e-3) / 1e12
    S0.close()
    net.close()
    out["roofline"] = {"bound": "mfma", "kernel": "network forward (k_net_features, k_conv x 3)",
                       "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s", "frac": tflops / 2500.0,
                       "traffic": None, "flop_per_launch": flop, "avg_launch_ms": fwd_ms,
                       "dtype": "bf16 (fp32 accumulate)"}
    print(json.dumps(out))


def bench_nonsym(args):
    """Nonsymmetric BoxMG (restriction from the transposed operator, coarse
    operators R A P) on a convection-diffusion operator: unit diffusion plus
    the upwind part of a recirculating flow of speed 300 on the 4095^2 grid,
    coarsest level 63^2.  One step = set-up + solve to the tolerance.  The
    roofline is that of the fine level's Gauss-Seidel sweep (two launches, each
    the two colours of the rows of one parity), timed with HIP events on the
    library's stream after the timed steps: per launch the stencil rows,
    right-hand side and new values of its half of the points (88 B each) and
    the iterate read once (8 B per point), 52 B per grid point."""
    import torch
    from paper_2502_05279_amd import boxmg, inputs

    dev = torch.device("cuda:0")
    n = int(args.workload.split("_")[1]) if args.workload != "cd_4095" else 4095
    beta = 300.0
    k = torch.from_numpy(inputs.constant_k(n)).to(dev)
    f = torch.from_numpy(inputs.uniform_source(n, 702)).to(dev)
    diff, rhs = boxmg.discretize(k, f)
    st = (diff + torch.from_numpy(inputs.upwind_convection(n, beta, "rotating")).to(dev)).contiguous()
    coarsest = args.coarsest or min(63, n)
    opts = dict(max_cycles=args.max_cycles, coarsest_n=coarsest)

    def step():
        S = boxmg.NSSolver(st, **opts)
        x, info = S.solve(rhs, tol=args.tol, raise_on_noconv=False)
        return S, x, info

    for _ in range(args.warmup):
        step()[0].close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k_ in range(args.steps):
        S, x, info = step()
        if k_ + 1 < args.steps:
            S.close()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the fine level's sweep, timed on the library's stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    ev0.record()
    for _ in range(reps):
        S.step(0, "smooth", 1)
    ev1.record()
    torch.cuda.synchronize()
    launch_ms = ev0.elapsed_time(ev1) / (2 * reps)
    S.close()
    bytes_per_launch = 52.0 * n * n
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    out = {
        "metric": f"fine DOF/s solved to {args.tol:g} rel. residual ({n}^2 convection-diffusion, nonsymmetric BoxMG)",
        "value": n * n / dt, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"cd_{n}", "n": n, "beta": beta, "flow": "rotating", "coarsest": coarsest,
                   "cycles": info["cycles"], "rho": info["rho"], "final_rel_res": info["rel_res"],
                   "converged": info["status"] == 0},
        "roofline": {"bound": "hbm", "kernel": "k_ns_gs_pair (fine level, the two colours of one row parity)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_ms": launch_ms, "bytes_per_launch": bytes_per_launch},
    }
    print(json.dumps(out))


def bench_block(args):
    """k right-hand sides on the jumping_4095 operator solved as one block: the
    fused passes run the tiles of all of them per launch and read the operator
    and weights about once.  One step = set-up of the hierarchy + the block
    solve of all k to the tolerance."""
    import torch
    from paper_2502_05279_amd import boxmg, inputs

    dev = torch.device("cuda:0")
    K = args.rhs
    p = workload(args.workload)
    n = p.n
    kk = torch.from_numpy(p.k).to(dev)
    stencil, _ = boxmg.discretize(kk, torch.from_numpy(p.f).to(dev))
    rhs = torch.stack([boxmg.discretize(kk, torch.from_numpy(f).to(dev))[1]
                       for f in inputs.extra_sources(n, K)])
    opts = dict(max_cycles=args.max_cycles, check_every=16,
                coarsest_n=args.coarsest or default_coarsest(args.workload, n))
    ws = {}

    def step(trace: bool):
        S = boxmg.Solver(stencil, workspace=ws.get("s"), **opts)
        ws["s"] = S.workspace
        B = boxmg.Block(S, K, workspace=ws.get("b"))
        ws["b"] = B.workspace
        if trace:
            B.trace_enable("pre", 0)
        x, infos = B.solve(rhs, tol=args.tol, raise_on_noconv=False)
        return S, B, x, infos

    for _ in range(args.warmup):
        S, B, _, _ = step(False)
        B.close()
        S.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launches, kms, kbytes, cyc, working = 0, 0.0, 0.0, 0, 0
    for _ in range(args.steps):
        S, B, x, infos = step(True)
        nl, ms, nb = B.trace_read()
        B.close()
        launches += nl
        kms += ms
        kbytes += nb
        cyc += sum(i["cycles"] for i in infos)
        working += max(i["cycles"] for i in infos)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n1 = S.level_n(1)
    S.close()
    # the library counts every launch with all k right-hand sides; launches
    # where some have stopped move less: count the operator and weights once per
    # working launch and the per-right-hand-side arrays once per cycle of each
    shared = 8.0 * (3 * n * n + 8 * n1 * n1)
    per_rhs = 8.0 * (3 * n * n + 2 * n1 * n1)
    assert abs(kbytes - launches * (shared + K * per_rhs)) <= 1e-9 * kbytes
    alg = working * shared + cyc * per_rhs
    avg_ms = kms / max(working, 1)
    achieved = alg / (kms * 1e-3) / 1e9
    out = {
        "metric": f"fine DOF/s solved to {args.tol:g} rel. residual ({n}^2, {K} right-hand sides "
                  "on one hierarchy)",
        "value": K * n * n / (dt / args.steps), "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}_rhs{K}", "n": n, "rhs": K, "tol": args.tol,
                   "cycles": [i["cycles"] for i in infos], "final_rel_res": max(i["rel_res"] for i in infos),
                   "converged": all(i["status"] == 0 for i in infos), "nu1": 2, "nu2": 1,
                   "precision": "fp64"},
        "roofline": {"bound": "hbm", "kernel": "pre", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "traffic_unit": "B/launch", "launches": launches, "working_launches": working,
                     "avg_launch_ms": avg_ms, "bytes_per_launch": alg / max(working, 1),
                     "bytes_per_point": alg / max(working, 1) / (n * n)},
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="jumping_4095")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-cycles", type=int, default=2000)
    ap.add_argument("--kernels", default="fused", choices=["fused", "basic"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32ir"],
                    help="fp64: FP64 V-cycles (double-FP64 below 16*tol); fp32ir: FP32 "
                         "V-cycles inside double-FP64 iterative refinement")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="with --precision fp32ir: also time the FP64 solve of the same "
                         "problem and report the difference of the two solutions")
    ap.add_argument("--cpu-baseline", choices=("solve", "full", "none"), default="solve",
                    help="solve: the oracle's whole solve once on all host cores; full: the "
                         "median of 3 on all cores and of 3 on one core; none: skip")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--coarsest", type=int, default=0,
                    help="points per side of the directly solved coarsest level (0 = the "
                         "workload's default: 63 on the jumping fields, 3 otherwise)")
    ap.add_argument("--refine-factor", type=int, default=None, metavar="F",
                    help="FP64: turn to double-FP64 refinement steps at F * tol (default: "
                         "the library's 16; 0 = never)")
    ap.add_argument("--graph", action="store_true",
                    help="plain FP64 cycles replayed from a captured HIP graph of two cycles")
    ap.add_argument("--square-tiles", type=int, default=0, metavar="N",
                    help="nine-point levels of at most N points per side run their fused "
                         "passes in square tiles (2^k - 1; 1 = none; 0 = the library's 511)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (a kernel of known traffic, to "
                         "calibrate hardware byte counters) and print the achieved GB/s")
    ap.add_argument("--params", default=None, help="learned_4095: network parameters (.npy)")
    ap.add_argument("--learned-n", type=int, default=4095)
    ap.add_argument("--smoother", choices=("point", "line"), default="point",
                    help="line: alternating zebra line relaxation (unfused cycle)")
    ap.add_argument("--rhs", type=int, default=1,
                    help="right-hand sides solved as one block on the workload's operator")
    ap.add_argument("--batch-tile-rows", type=int, default=0,
                    help="batch_512: tile height of every level instead of the autotuner's")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported: the solver "
              "is built for a single MI355X (see the design notes for how it would shard).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_05279_amd import boxmg

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    if args.workload == "batch_512":
        return bench_batch(args)
    if args.workload.startswith("cd_"):
        return bench_nonsym(args)
    if args.workload == "learned_4095":
        return bench_learned(args)
    if args.rhs > 1:
        return bench_block(args)
    if args.copy_probe:
        a = torch.ones(args.copy_probe << 17, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        print(json.dumps({"copy_probe_bytes": 2 * a.numel() * 8, "seconds": dt,
                          "GB_per_s": 2 * a.numel() * 8 / dt / 1e9}))
        return
    p = workload(args.workload)
    n = p.n
    k = torch.from_numpy(p.k).to(dev)
    f = torch.from_numpy(p.f).to(dev)
    stencil, rhs = boxmg.discretize(k, f)
    kern = boxmg.BMG_KERNELS_FUSED if args.kernels == "fused" else boxmg.BMG_KERNELS_BASIC
    prec = boxmg.BMG_FP32_IR if args.precision == "fp32ir" else boxmg.BMG_FP64
    line = args.smoother == "line"
    coarsest = args.coarsest or default_coarsest(args.workload, n)
    opts = dict(max_cycles=args.max_cycles, kernels=kern, check_every=16, precision=prec,
                smoother=boxmg.BMG_SMOOTH_LINE if line else boxmg.BMG_SMOOTH_POINT,
                coarsest_n=coarsest, square_tiles_below_n=args.square_tiles)
    if args.refine_factor is not None:
        opts["refine_factor"] = args.refine_factor
    if args.graph:
        opts["graph_mode"] = 1
    tclass = "pre" if args.kernels == "fused" and not line else "smooth"
    if prec == boxmg.BMG_FP32_IR:
        tclass = "resnorm"     # the FP64 outer residual (accurate, 64 B per point)
    elif tclass == "pre":
        # FP64 V(2,1) on the five-point fine level: the fine post pass of each
        # plain cycle runs with the next cycle's fine pre pass (k_postpre)
        tclass = "postpre"

    def step(trace: bool):
        S = boxmg.Solver(stencil, **opts)
        if trace:
            S.trace_enable(tclass, 0)
        x, info = S.solve(rhs, tol=args.tol, raise_on_noconv=False)
        return S, x, info

    for _ in range(args.warmup):
        step(False)[0].close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    launches, kms, kbytes = 0, 0.0, 0.0
    for _ in range(args.steps):
        S, x, info = step(True)
        nl, ms, nb = S.trace_read()
        S.close()
        launches += nl
        kms += ms
        kbytes += nb
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    info = infos[-1]
    ms_step = dt * 1e3 / args.steps
    bpl = kbytes / max(launches, 1)                     # algorithmic bytes per launch
    # a solve's last batch of cycles ends in launches that return at once (the
    # stop flag is set); the fine pre pass runs once per cycle, so its working
    # launches are the cycles, and their average includes those few microseconds
    working = launches
    if tclass == "pre":
        working = min(launches, sum(i["cycles"] for i in infos))
    if tclass == "postpre":
        # one per plain cycle: up to the first residual at or below 16 tol,
        # where the solve turns to double-FP64 refinement steps
        def plain(i):
            h = i["history"]
            return next((k + 1 for k, v in enumerate(h) if v <= 16 * args.tol), len(h))
        working = min(launches, sum(plain(i) for i in infos))
    avg_ms = kms / max(working, 1)
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if working else None
    # the survey's counting rule for a fused pass: the smoother's stream (stencil,
    # b, u read, u written: 48 B per fine point) once, plus the interpolation
    # weights (16), e_c and b_c (2 each) it reads or writes: 68 B per fine point
    # for k_postpre; the library's count (bpl) adds the second iterate written
    # (u_k, 8) and the zeroed coarse iterate (2): 78
    survey_bpl = None
    if tclass == "postpre":
        survey_bpl = 68.0 * n * n
    if survey_bpl is not None and working:
        achieved_lib = achieved
        achieved = survey_bpl / (avg_ms * 1e-3) / 1e9
    traffic = None
    if tclass == "pre" and args.kernels == "fused":
        traffic = measured_traffic(f"{args.workload} {args.precision} pre", boxmg.tile_rows_get(n))
    if tclass == "postpre":
        traffic = measured_traffic(f"{args.workload} {args.precision} postpre")
    # the headline metric names the 4095^2 workload; other sizes and tolerances
    # say their own
    metric = METRIC if (n == 4095 and args.tol == 1e-10) else \
        f"fine DOF/s solved to {args.tol:g} rel. residual ({n}^2); smoother HBM GB/s vs peak"
    extra = {}
    if line:
        metric = f"fine DOF/s solved to {args.tol:g} rel. residual ({n}^2, line relaxation)"
    if prec == boxmg.BMG_FP32_IR:
        metric = f"fine DOF/s solved to {args.tol:g} rel. residual ({n}^2, FP32 V-cycle in FP64 refinement)"
        if args.compare_fp64:
            o64 = dict(opts, precision=boxmg.BMG_FP64)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            S64 = boxmg.Solver(stencil, **o64)
            x64, info64 = S64.solve(rhs, tol=args.tol, raise_on_noconv=False)
            torch.cuda.synchronize()
            t64 = time.perf_counter() - t1
            S64.close()
            d = (x - x64)
            extra = {"fp64_ms_per_solve": t64 * 1e3, "fp64_cycles": info64["cycles"],
                     "fp64_final_rel_res": info64["rel_res"],
                     "rel_diff_to_fp64_2norm": float(d.norm() / x64.norm()),
                     "rel_diff_to_fp64_inf": float(d.abs().max() / x64.abs().max())}
    out = {
        "metric": metric,
        "value": n * n / (dt / args.steps),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == boxmg.BMG_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "dof": n * n, "tol": args.tol,
                   "cycles": info["cycles"], "final_rel_res": info["rel_res"],
                   "converged": info["status"] == 0, "rho": info["rho"],
                   "coarsest": coarsest, "floor_est": info["floor_est"],
                   "setup_ms": float(np.mean([i["t_setup_ms"] for i in infos])),
                   "solve_ms": float(np.mean([i["t_solve_ms"] for i in infos])),
                   "kernels": "basic" if line else args.kernels, "smoother": args.smoother,
                   "nu1": 2, "nu2": 1, "precision": args.precision, "graph_mode": int(args.graph),
                   **extra},
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES.get(tclass, tclass), "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": traffic, "traffic_unit": "B/launch",
                     "launches": launches, "working_launches": working, "avg_launch_ms": avg_ms,
                     "bytes_per_launch": survey_bpl or bpl, "bytes_per_point": (survey_bpl or bpl) / (n * n)},
    }
    if survey_bpl is not None and working:
        out["roofline"]["counting"] = ("achieved/frac: 68 B per fine point (smoother stream 48 once, weights 16, "
                                       "e_c 2, b_c 2); achieved_all_arrays/frac_all_arrays: 78 B per fine "
                                       "point, every array the pass touches once (adds u_k written 8, u_c "
                                       "zeroed 2)")
        out["roofline"]["achieved_all_arrays"] = achieved_lib
        out["roofline"]["frac_all_arrays"] = achieved_lib / HBM_PEAK_GBS
    if not args.no_cpu_baseline and args.cpu_baseline != "none":
        out["cpu_baseline"] = cpu_baseline(p, coarsest, args.tol, args.cpu_baseline == "full")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
