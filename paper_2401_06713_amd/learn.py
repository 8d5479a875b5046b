"""Training the parameter predictor from sweeps the method runs itself.

The paper picks (palette %, alpha) by sweeping a grid on training graphs,
scoring each point with a bi-objective (Eq. 7: beta * colours + (1 - beta) *
|E_c|) for several values of beta, and training a regressor that is given
the graph and beta (Sec. VI, Steps 1-6).  Here:

* sweep: every training instance is coloured with the fixed parameters
  (f = 0.125, alpha = 2) and at every grid point; each run records the colour
  count, the largest per-iteration |E_c| (the memory driver) and its time;
* label, per beta: J = beta * C / C_fixed + (1 - beta) * E / E_fixed (the
  raw sum of Eq. 7 mixes units, hence the normalisation) minimised over the
  grid points with C <= (1 - margin) C_fixed; the fixed point itself is
  always a candidate;
* rows: the features of every iteration of the fixed run (iteration l's
  vertex set is the set of vertices whose colour id is at least that
  iteration's palette offset) followed by beta, each with its instance's
  label for that beta;
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
# Network parameters trained by `python -m paper_2401_06713_amd.learn --train 1000 --steps 4000
# --margin 0.01` (sweeps over 1000 instances, n log-uniform in [1e3, 1e5], q in 16..96, labels for
# beta 0.1 .. 0.9); predictor.json beside it holds the held-out evaluation and the accepted beta.
PREDICTOR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "predictor.npy")
# The grid: palettes 4%-17% of the vertices and alpha 1-3 (the paper sweeps
# 1%-20% and 0.5-4.5, Sec. VI).  Smaller palettes with longer lists cost
# tens of times the fixed run's edges, and alpha below 1 is outside the
# predictor's output range [1, 4].
GRID_F = (0.04, 0.06, 0.08, 0.09, 0.10, 0.11, 0.125, 0.14, 0.17)
GRID_A = (1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0)
GROUP_STRINGS = 2_000_000  # strings per batched sweep call


@dataclass
class Run:
    frac: float
    alpha: float
    colors: int
    max_edges: int
    ms: float
    peak_bytes: int


def squash(o):
    """Network outputs -> (palette fraction, list multiplier): the map the
    library applies to the network's outputs, restated for labels and
    reports."""
    o = np.asarray(o, dtype=np.float64)
    return 0.01 + 0.24 / (1 + np.exp(-o[..., 0])), 1.0 + 3.0 / (1 + np.exp(-o[..., 1]))


def unsquash(frac, alpha):
    """(palette fraction, list multiplier) -> network targets (the inverse
    of squash), clipped inside the open ranges."""
    u = np.clip((np.asarray(frac, dtype=np.float64) - 0.01) / 0.24, 1e-3, 1 - 1e-3)
    w = np.clip((np.asarray(alpha, dtype=np.float64) - 1.0) / 3.0, 1e-3, 1 - 1e-3)
    return np.stack([np.log(u / (1 - u)), np.log(w / (1 - w))], axis=-1)


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


def label(runs: list[Run], fixed: Run, beta: float, margin: float = 0.0) -> Run:
    ok = [r for r in runs if r.colors <= (1.0 - margin) * fixed.colors] + [fixed]
    return min(ok, key=lambda r: objective(r, fixed, beta))


BETAS = (0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9)


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


def iteration_sets(col: np.ndarray, frac: float):
    """Per-iteration vertex sets of a finished fixed-parameter colouring,
    rebuilt from its colours: iteration l uses the colour ids
    [offset_l, offset_l + P_l) with P_l = max(1, ceil(frac m_l)), so its
    vertex set is the vertices whose colour is at least offset_l."""
    sets = []
    off, m = 0, col.shape[0]
    while m > 0:
        ids = np.nonzero(col >= off)[0].astype(np.int32)
        assert ids.size == m
        sets.append(ids)
        off += max(1, math.ceil(frac * m))
        m = int((col >= off).sum())
    return sets


def sweep(cfgs, betas=BETAS, grid_f=GRID_F, grid_a=GRID_A, margin: float = 0.0, log=print):
    """Returns (input rows: features and beta, targets rows, per-instance records).

    All training instances sit in one batch handle: the fixed run and every
    grid point are one batched colouring each; per-instance colour counts
    and largest |E_c| come from the instance statistics."""
    insts = [wl.make(c) for c in cfgs]
    fixed, runs, cols = [None] * len(cfgs), [[] for _ in cfgs], [None] * len(cfgs)
    # groups of at most GROUP_STRINGS strings: at the grid's small palettes and
    # long lists the bucket matrices take about m T^2 / (8 f) bytes
    groups, cur, size = [], [], 0
    for i, c in enumerate(cfgs):
        if cur and size + c.n > GROUP_STRINGS:
            groups.append(cur)
            cur, size = [], 0
        cur.append(i)
        size += c.n
    if cur:
        groups.append(cur)
    for gi, idx in enumerate(groups):
        seeds = [cfgs[i].seed for i in idx]
        rels = [cfgs[i].relation for i in idx]
        with pk.PicassoBatch([(insts[i][0], insts[i][1], cfgs[i].q) for i in idx]) as hb:
            hb.set_option(pk.OPT_MEM_BUDGET, 1)  # count the edges, write no CSR: the sweep needs only counts
            t = time.perf_counter()
            nc_fixed, gcols = hb.color_batch(seeds, FIXED[0], FIXED[1], rels)
            ms_fixed = (time.perf_counter() - t) * 1e3
            ist = hb.instance_stats()
            for k, i in enumerate(idx):
                fixed[i] = Run(*FIXED, int(nc_fixed[k]), ist[k]["max_edges"], ms_fixed, 0)
                cols[i] = gcols[k]
            for f in grid_f:
                for a in grid_a:
                    t = time.perf_counter()
                    nc, _ = hb.color_batch(seeds, f, a, rels)
                    ms = (time.perf_counter() - t) * 1e3
                    ist = hb.instance_stats()
                    for k, i in enumerate(idx):
                        runs[i].append(Run(f, a, int(nc[k]), ist[k]["max_edges"], ms, 0))
        if log:
            log(f"sweep: group {gi + 1}/{len(groups)} ({len(idx)} instances) done")
    X, Y, recs = [], [], []
    for i, cfg in enumerate(cfgs):
        x, z = insts[i]
        with pk.Picasso(x, z, cfg.q) as h:
            feats = np.array([h.features(cfg.seed, k + 1, ids, cfg.relation)
                              for k, ids in enumerate(iteration_sets(cols[i], FIXED[0]))], dtype=np.float64)
        best = {}
        for beta in betas:
            b = label(runs[i], fixed[i], beta, margin)
            best[beta] = asdict(b)
            X.append(np.concatenate([feats, np.full((len(feats), 1), beta)], axis=1))
            Y.append(np.repeat(unsquash(b.frac, b.alpha)[None, :], len(feats), axis=0))
        recs.append({"config": asdict(cfg), "fixed": asdict(fixed[i]), "best": best,
                     "runs": [asdict(r) for r in runs[i]]})
    if log:
        for beta in betas:
            gain = np.mean([objective(label(rr, ff, beta, margin), ff, beta) for rr, ff in zip(runs, fixed)])
            log(f"sweep: {len(cfgs)} instances, beta {beta}: mean best J {gain:.3f} (fixed = 1)")
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


def evaluate(mlp: pk.Mlp, cfgs, betas=(0.5,), judge: bool = False, repeats: int = 1, log=None):
    """Per instance: fixed vs learned colours, largest |E_c|, time, peak
    bytes, for each beta.

    Each method runs on a handle of its own: one untimed call (which sizes
    the handle's buffers), then `repeats` timed calls, the fastest kept, so
    the peak counts only that method's buffers and no time includes device
    allocation.  The learned run consults the network every iteration, so it
    does not use the tail kernel; the fixed run is timed the same way
    (`fixed`), and with the tail kernel as well (`fixed_tail_ms`)."""
    def timed(h, call):
        call()  # sizes the buffers
        best, res = float("inf"), None
        for _ in range(max(1, repeats)):
            t = time.perf_counter()
            res = call()
            best = min(best, (time.perf_counter() - t) * 1e3)
        return best, res

    out = {float(b): [] for b in betas}
    for cfg in cfgs:
        x, z = wl.make(cfg)
        with pk.Picasso(x, z, cfg.q) as h:
            tail_ms, _ = timed(h, lambda: h.color(cfg.seed, *FIXED, cfg.relation))
        with pk.Picasso(x, z, cfg.q) as h:
            h.set_option(pk.OPT_TAIL, 0)
            ms, (nc, _) = timed(h, lambda: h.color(cfg.seed, *FIXED, cfg.relation))
            st = h.stats()
            fixed = Run(*FIXED, nc, st["max_edges"], ms, st["peak_device_bytes"])
        for beta in betas:
            with pk.Picasso(x, z, cfg.q) as h:
                h.set_option(pk.OPT_LEARNED_JUDGE, int(judge))
                ms, (nc, _, sched) = timed(h, lambda: h.color_learned(mlp, cfg.seed, cfg.relation, beta))
                st = h.stats()
            learned = Run(float(sched[0, 0]), float(sched[0, 1]), nc, st["max_edges"], ms, st["peak_device_bytes"])
            out[float(beta)].append({"n": cfg.n, "q": cfg.q, "seed": cfg.seed, "fixed": asdict(fixed),
                                     "fixed_tail_ms": tail_ms, "learned": asdict(learned),
                                     "J_learned": objective(learned, fixed, beta), "schedule": sched.tolist(),
                                     "judged": st["judged"], "csr_refills": st["csr_refills"],
                                     "library_ms": st["ms_total"],
                                     "jp_rounds": [it["jp_rounds"] for it in st["iters"][:st["n_iters"]]]})
        if log:
            log(f"evaluate: {cfg.name} fixed {fixed.colors} colours; learned " +
                ", ".join(f"beta {b}: {out[float(b)][-1]['learned']['colors']}" for b in betas))
    return out


def summarize(res: list) -> dict:
    """Mean ratios learned / fixed over the evaluated instances."""
    def mean(key):
        return float(np.mean([r["learned"][key] / r["fixed"][key] for r in res]))

    return {"count": len(res), "mean_J_learned": float(np.mean([r["J_learned"] for r in res])),
            "colors_ratio": mean("colors"), "max_edges_ratio": mean("max_edges"), "ms_ratio": mean("ms"),
            "ms_ratio_vs_fixed_with_tail": float(np.mean([r["learned"]["ms"] / r["fixed_tail_ms"] for r in res])),
            "peak_bytes_ratio": mean("peak_bytes"),
            "colors_ratio_max": float(max(r["learned"]["colors"] / r["fixed"]["colors"] for r in res)),
            "instances_with_fewer_or_equal_colours": int(sum(r["learned"]["colors"] <= r["fixed"]["colors"]
                                                              for r in res))}


def heldout_instances(count: int, n: int, q: int, pI: float, seed: int = 7_000_000):
    """Held-out instances: n strings on q qubits, identity with probability
    pI and X/Y/Z equal; anticommute relation; instance i uses seed seed + i."""
    r = (1 - pI) / 3
    return [wl.Config(f"heldout[{i}]", n, q, (pI, r, r, r), seed + i, FIXED[0], FIXED[1], 0) for i in range(count)]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train", type=int, default=1000, help="training instances")
    ap.add_argument("--n-lo", type=int, default=1000)
    ap.add_argument("--n-hi", type=int, default=100_000)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--betas", type=float, nargs="+", default=list(BETAS), help="labels for these beta values")
    ap.add_argument("--margin", type=float, default=0.0,
                    help="labels need C <= (1 - margin) C_fixed (else the fixed parameters)")
    ap.add_argument("--grid-f", type=float, nargs="+", default=list(GRID_F))
    ap.add_argument("--grid-a", type=float, nargs="+", default=list(GRID_A))
    ap.add_argument("--eval-betas", type=float, nargs="+", default=[0.1, 0.5, 0.9])
    ap.add_argument("--heldout", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=3, help="timed calls per method and instance (fastest kept)")
    ap.add_argument("--heldout-n", type=int, default=500_000)
    ap.add_argument("--heldout-q", type=int, default=96)
    ap.add_argument("--heldout-pi", type=float, default=0.75)
    ap.add_argument("--out", default="predictor")
    ap.add_argument("--params", default=None, help="evaluate these saved network parameters (.npy) only")
    args = ap.parse_args()
    say = lambda *a: print(*a, flush=True)  # noqa: E731
    if args.params:
        mlp, loss, rows, sweep_s, n_train = pk.Mlp(np.load(args.params)), None, 0, 0.0, 0
    else:
        cfgs = training_instances(args.train, n_lo=args.n_lo, n_hi=args.n_hi)
        t = time.perf_counter()
        X, Y, recs = sweep(cfgs, args.betas, tuple(args.grid_f), tuple(args.grid_a), args.margin, log=say)
        sweep_s = time.perf_counter() - t
        with open(args.out + "_sweep.json", "w") as f:
            json.dump(recs, f)
        mlp, loss = train(X, Y, steps=args.steps, log=say)
        rows, n_train = int(X.shape[0]), len(cfgs)
        np.save(args.out + ".npy", mlp.get_params())
    held = heldout_instances(args.heldout, args.heldout_n, args.heldout_q, args.heldout_pi)
    res = evaluate(mlp, held, args.eval_betas, repeats=args.repeats, log=say)
    summary = {
        "betas": args.betas, "margin": args.margin, "grid_f": args.grid_f, "grid_a": args.grid_a,
        "train_instances": n_train, "n_range": [args.n_lo, args.n_hi], "rows": rows, "final_loss": loss,
        "sweep_seconds": sweep_s,
        "heldout": {"count": len(held), "n": args.heldout_n, "q": args.heldout_q, "pI": args.heldout_pi,
                    "by_beta": {str(b): {**summarize(r), "instances": r} for b, r in res.items()}},
    }
    # the most colour-weighted beta at which the learned parameters use no
    # more colours than the fixed ones on every held-out instance, in less
    # time (against the fixed run with its tail kernel) and less device memory
    ok = [b for b, r in res.items()
          if summarize(r)["colors_ratio_max"] <= 1.0 and summarize(r)["ms_ratio_vs_fixed_with_tail"] < 1.0
          and summarize(r)["peak_bytes_ratio"] < 1.0]
    summary["acceptance_beta"] = max(ok) if ok else None
    with open(args.out + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    for b, r in res.items():
        say(f"held-out beta {b}:", json.dumps(summarize(r)))
    if not args.params:
        say("saved", os.path.abspath(args.out + ".npy"))


if __name__ == "__main__":
    main()
