"""Training and use of the learned interpolation (all arithmetic in the HIP
library; this module only schedules samples and moves arrays).

Training data are the operators of the levels with 31 to 255 points per side
of BoxMG hierarchies built on seeded coefficient fields; each sample is one
two-grid cycle on a level operator from a random residual, and the network
minimises the mean residual reduction ||r3||^2 / ||r0||^2 with Adam.  (Levels
of 7 and 15 points, where a coarse grid point stands for a quarter of the
domain, made the training diverge; the network corrects the weights of levels
of 31 points and more.)

    python -m paper_2502_05279_amd.learned train --fields 1000 --epochs 6 --lr 1e-4 \
        --out paper_2502_05279_amd/data/learned_p.npy
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import boxmg, inputs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "data", "learned_p.npy")


def level_stencils(k: np.ndarray, f: np.ndarray, device="cuda:0", min_n: int = 7, max_n: int = 1 << 15):
    """The operators of a BoxMG hierarchy's levels (min_n <= n <= max_n) as
    [n][n][K] device tensors, finest first."""
    st, _ = boxmg.discretize(torch.from_numpy(k).to(device), torch.from_numpy(f).to(device))
    S = boxmg.Solver(st)
    out = []
    for lvl in range(S.nlev):
        if min_n <= S.level_n(lvl) <= max_n:
            out.append(S.export(lvl, "stencil"))
    S.close()
    return out


def training_set(nfields: int, n: int = 255, seed0: int = 10_000, block: int = 16,
                 lo: float = -4.0, hi: float = 4.0, device="cuda:0", min_n: int = 7, max_n: int = 1 << 15):
    samples = []
    for s in range(nfields):
        p = inputs.learned_train_field(seed0 + s, n, block, lo, hi)
        samples.extend(level_stencils(p.k, p.f, device, min_n, max_n))
    return samples


class Trainer:
    """Adam on the two-grid loss over a list of level operators."""

    def __init__(self, net: boxmg.Net, inner_tol: float = 1e-8, inner_max: int = 30, coarsest: int = 15):
        self.net = net
        self.inner_tol = inner_tol
        self.inner_max = inner_max
        self.coarsest = coarsest    # the inner coarse solves' direct level (at most the sample's coarse level)
        self._ws = None

        self.skipped = 0

    def sample_loss(self, st: torch.Tensor, seed: int):
        """Loss of one sample (its gradient added to the network's sum), or
        None when the operator-induced weights of the levels below the learned
        one break down on the coarse operator (the sample is skipped)."""
        n = st.shape[0]
        need = boxmg.workspace_bytes(n, st.shape[2], coarsest_n=min(self.coarsest, (n - 1) // 2))
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 1 << 20), dtype=torch.uint8, device=st.device)
        try:
            S = boxmg.Solver(st, workspace=self._ws, interp=boxmg.BMG_INTERP_LEARNED, learned_levels=1,
                             net=self.net, coarsest_n=min(self.coarsest, (n - 1) // 2))
        except boxmg.BoxMGError as e:
            if e.status != boxmg.BMG_EBREAKDOWN:
                raise
            self.skipped += 1
            return None
        r0 = torch.from_numpy(inputs.residual_probe(n, seed)).to(st.device)
        loss, _ = self.net.twogrid(S, r0, self.inner_tol, self.inner_max)
        S.close()
        return loss

    def step(self, batch, seeds, lr: float):
        self.net.zero_grad()
        losses = [v for v in (self.sample_loss(st, sd) for st, sd in zip(batch, seeds)) if v is not None]
        if not losses:
            return None
        self.net.adam(lr, scale=1.0 / len(losses))
        return float(np.mean(losses))

    def mean_loss(self, samples, seed0: int) -> float:
        self.net.zero_grad()
        v = [x for x in (self.sample_loss(st, seed0 + t) for t, st in enumerate(samples)) if x is not None]
        return float(np.mean(v)) if v else float("nan")


def train(fields: int = 2000, epochs: int = 1, batch: int = 16, lr: float = 1e-3, n: int = 255,
          seed: int = 501, max_minutes: float | None = None, coarsest: int = 15, min_n: int = 31,
          max_n: int = 1 << 15, log=print):
    net = boxmg.Net(inputs.net_init(seed), max_n=n, train=True)
    tr = Trainer(net, coarsest=coarsest)
    samples = training_set(fields, n, min_n=min_n, max_n=max_n)
    held = training_set(8, n, seed0=90_000, min_n=min_n, max_n=max_n)
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    hist = {"held_out": [tr.mean_loss(held, 123_000)], "train": []}
    log(json.dumps({"samples": len(samples), "held_out_loss": hist["held_out"][0]}))
    step = 0
    for ep in range(epochs):
        order = rng.permutation(len(samples))
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            loss = tr.step([samples[t] for t in idx], [1_000_000 * (ep + 1) + int(t) for t in idx], lr)
            if loss is not None:
                hist["train"].append(loss)
            step += 1
            if step % 50 == 0:
                log(json.dumps({"epoch": ep, "step": step, "loss": float(np.mean(hist["train"][-50:])),
                                "skipped": tr.skipped, "s": round(time.perf_counter() - t0, 1)}))
            if max_minutes and time.perf_counter() - t0 > 60 * max_minutes:
                break
        hist["held_out"].append(tr.mean_loss(held, 123_000))
        log(json.dumps({"epoch": ep, "held_out_loss": hist["held_out"][-1]}))
        if max_minutes and time.perf_counter() - t0 > 60 * max_minutes:
            break
    return net, hist


def load_params(path: str = DEFAULT_PARAMS) -> np.ndarray:
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.size != boxmg.NET_PARAMS:
        raise ValueError(f"{path}: expected {boxmg.NET_PARAMS} float32 parameters")
    return p


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--fields", type=int, default=2000)
    t.add_argument("--epochs", type=int, default=1)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=501)
    t.add_argument("--max-minutes", type=float, default=None)
    t.add_argument("--coarsest", type=int, default=15)
    t.add_argument("--min-n", type=int, default=31)
    t.add_argument("--max-n", type=int, default=1 << 15)
    t.add_argument("--out", default=DEFAULT_PARAMS)
    a = ap.parse_args()
    if a.cmd == "train":
        net, hist = train(a.fields, a.epochs, a.batch, a.lr, seed=a.seed, max_minutes=a.max_minutes,
                          coarsest=a.coarsest, min_n=a.min_n, max_n=a.max_n, log=lambda s: print(s, flush=True))
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.save(a.out, net.params())
        print(json.dumps({"saved": a.out, "held_out": hist["held_out"]}), flush=True)


if __name__ == "__main__":
    main()
