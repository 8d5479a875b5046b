"""Training the parameter predictor from sweeps the method runs itself.

The paper picks (palette %, alpha) by sweeping a grid on training graphs,
scoring each point with a bi-objective (Eq. 7: beta * colours + (1 - beta) *
|E_c|) and training a regressor on the argmins (Sec. VI).  Here:

* sweep: every training instance is coloured with the fixed parameters
  (f = 0.125, alpha = 2) and at every grid point; each run records the colour
  count, the largest per-iteration |E_c| (the memory driver) and its time;
* label: J = beta * C / C_fixed + (1 - beta) * E / E_fixed (the raw sum of
  Eq. 7 mixes units, hence the normalisation) minimised over the grid points
  with C <= C_fixed; the fixed point itself is always a candidate;
* rows: the features of every iteration of the fixed run (iteration l's
  vertex set is the set of vertices whose colour id is at least that
  iteration's palette offset), each with its instance's label;
* training: mini-batch Adam on the device network (Mlp.train_step).

All colouring runs, features and training steps go through libpicasso.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time
from dataclasses import asdict, dataclass

import numpy as np

import paper_2401_06713_amd as pk
from paper_2401_06713_amd import workloads as wl

FIXED = (0.125, 2.0)
GRID_F = (0.02, 0.04, 0.06, 0.08, 0.10, 0.125, 0.15, 0.20, 0.25)
GRID_A = (1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0)


@dataclass
class Run:
    frac: float
    alpha: float
    colors: int
    max_edges: int
    ms: float
    peak_bytes: int


def run_once(h: pk.Picasso, seed: int, frac: float, alpha: float, rel: int) -> Run:
    t = time.perf_counter()
    nc, col = h.color(seed, frac, alpha, rel)
    ms = (time.perf_counter() - t) * 1e3
    st = h.stats()
    return Run(frac, alpha, nc, st["max_edges"], ms, st["peak_device_bytes"])


def iteration_features(h: pk.Picasso, col: np.ndarray, stats: dict, seed: int, rel: int) -> np.ndarray:
    rows = []
    for k, it in enumerate(stats["iters"]):
        ids = np.nonzero(col >= it["offset"])[0].astype(np.int32)
        if ids.size == 0:
            break
        rows.append(h.features(seed, k + 1, ids, rel))
    return np.array(rows, dtype=np.float64)


def objective(r: Run, fixed: Run, beta: float) -> float:
    return beta * r.colors / fixed.colors + (1 - beta) * r.max_edges / max(fixed.max_edges, 1)


def label(runs: list[Run], fixed: Run, beta: float) -> Run:
    ok = [r for r in runs if r.colors <= fixed.colors] + [fixed]
    return min(ok, key=lambda r: objective(r, fixed, beta))


def training_instances(count: int, seed: int = 10**6, n_lo: int = 1000, n_hi: int = 100_000):
    """n log-uniform in [n_lo, n_hi], q uniform in {16..96}, pI uniform in
    [0.5, 0.85] with X/Y/Z equal; anticommute relation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        q = int(rng.integers(16, 97))
        pI = float(rng.uniform(0.5, 0.85))
        r = (1 - pI) / 3
        out.append(wl.Config(f"train[{i}]", n, q, (pI, r, r, r), seed + i, FIXED[0], FIXED[1], 0))
    return out


def sweep(cfgs, beta: float = 0.5, grid_f=GRID_F, grid_a=GRID_A, log=print):
    """Returns (features rows, targets rows, per-instance records)."""
    X, Y, recs = [], [], []
    for i, cfg in enumerate(cfgs):
        x, z = wl.make(cfg)
        with pk.Picasso(x, z, cfg.q) as h:
            nc, col = h.color(cfg.seed, *FIXED, cfg.relation)
            st = h.stats()
            fixed = Run(*FIXED, nc, st["max_edges"], st["ms_total"], st["peak_device_bytes"])
            feats = iteration_features(h, col, st, cfg.seed, cfg.relation)
            runs = [run_once(h, cfg.seed, f, a, cfg.relation) for f in grid_f for a in grid_a]
        best = label(runs, fixed, beta)
        X.append(feats)
        Y.append(np.repeat(pk.unsquash(best.frac, best.alpha)[None, :], len(feats), axis=0))
        recs.append({"config": asdict(cfg), "fixed": asdict(fixed), "best": asdict(best)})
        if log:
            log(f"sweep {i + 1}/{len(cfgs)} n={cfg.n} q={cfg.q}: fixed C={fixed.colors} E={fixed.max_edges}; "
                f"best f={best.frac} a={best.alpha} C={best.colors} E={best.max_edges}")
    return np.concatenate(X), np.concatenate(Y), recs


def train(X, Y, steps: int = 2000, batch: int = 256, lr: float = 3e-3, seed: int = 0, mlp: pk.Mlp | None = None,
          log=print):
    rng = np.random.default_rng(seed)
    mlp = mlp or pk.Mlp(seed=seed)
    X = X.astype(np.float32)
    Y = Y.astype(np.float32)
    loss = float("nan")
    for s in range(steps):
        idx = rng.integers(0, X.shape[0], min(batch, X.shape[0]))
        loss = mlp.train_step(X[idx], Y[idx], lr)
        if log and (s % 500 == 0 or s == steps - 1):
            log(f"train step {s}: loss {loss:.4f}")
    return mlp, loss


def evaluate(mlp: pk.Mlp, cfgs, beta: float = 0.5):
    """Per instance: fixed vs learned colours, largest |E_c|, time, peak bytes."""
    out = []
    for cfg in cfgs:
        x, z = wl.make(cfg)
        with pk.Picasso(x, z, cfg.q) as h:
            h.color(cfg.seed, *FIXED, cfg.relation)  # warm-up
            fixed = run_once(h, cfg.seed, *FIXED, cfg.relation)
            t = time.perf_counter()
            nc, _, sched = h.color_learned(mlp, cfg.seed, cfg.relation)
            ms = (time.perf_counter() - t) * 1e3
            st = h.stats()
        learned = Run(float(sched[0, 0]), float(sched[0, 1]), nc, st["max_edges"], ms, st["peak_device_bytes"])
        out.append({"n": cfg.n, "q": cfg.q, "fixed": asdict(fixed), "learned": asdict(learned),
                    "J_learned": objective(learned, fixed, beta)})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train", type=int, default=60, help="training instances")
    ap.add_argument("--n-hi", type=int, default=100_000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--beta", type=float, default=0.5)
    ap.add_argument("--out", default="predictor")
    args = ap.parse_args()
    cfgs = training_instances(args.train, n_hi=args.n_hi)
    X, Y, recs = sweep(cfgs, args.beta)
    mlp, loss = train(X, Y, steps=args.steps)
    np.save(args.out + ".npy", mlp.get_params())
    with open(args.out + ".json", "w") as f:
        json.dump({"beta": args.beta, "rows": int(X.shape[0]), "final_loss": loss, "sweep": recs}, f, indent=1)
    print("saved", os.path.abspath(args.out + ".npy"))


if __name__ == "__main__":
    main()
