"""Write stored oracle results for the full-size workloads.

Calls only the CPU oracle (oracle/) and the seeded input generator; the
HIP path is never involved.  Each JSON file holds the colour count, the
SHA-256 of the little-endian int32 colour array and the per-iteration sizes.

    python tests/golden/make_golden.py C2 [seed ...]
    python tests/golden/make_golden.py L 7000000     # the first held-out instance
    python tests/golden/make_golden.py C3 [workers]   # the 512-instance batch
    python tests/golden/make_golden.py C4 [workers]   # n = 2,000,000, q = 128, seed 0
    python tests/golden/make_golden.py C2dyn [divisor] # C2 seed 0, dynamic colourer (round form),
                                                     # with the sequential Alg. 2 colour count beside it
    python tests/golden/make_golden.py Llearned [beta] # the first held-out instance coloured with the
                                                     # stored network's parameters (FP64 twin), at the
                                                     # beta its evaluation accepted unless given

The C4 run colours each iteration from its colour classes (the oracle's
edge-free mode: its conflict graph, 3.6e9 edges in iteration 1, does not fit
a host), then counts each iteration's conflict edges colour slice by colour
slice in worker processes.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2401_06713_amd import workloads as wl  # noqa: E402

CONFIGS = {"C1": wl.C1, "C2": wl.C2, "C4": wl.C4, "L": wl.LHELD0}


def _batch_one(i):
    cfg = wl.batch_instances()[i]
    x, z = wl.make(cfg)
    t = time.time()
    nc, col, st = oracle.color(x, z, cfg.q, cfg.seed, cfg.frac, cfg.alpha, cfg.relation)
    return {
        "index": i,
        "n": cfg.n,
        "q": cfg.q,
        "pI": cfg.probs[0],
        "seed": cfg.seed,
        "relation": cfg.relation,
        "n_colors": nc,
        "n_iters": len(st),
        "colors_sha256": hashlib.sha256(np.ascontiguousarray(col, dtype="<i4").tobytes()).hexdigest(),
        "oracle_seconds": round(time.time() - t, 2),
    }


def batch_main(workers):
    from multiprocessing import Pool

    oracle.build(force=False)
    cfgs = wl.batch_instances()
    count = len(cfgs)
    # largest first, so the pool ends evenly
    order = sorted(range(count), key=lambda i: -cfgs[i].n)
    with Pool(workers) as pool:
        recs = []
        for k, r in enumerate(pool.imap_unordered(_batch_one, order)):
            recs.append(r)
            if k % 32 == 0:
                print(f"{k + 1}/{count}", flush=True)
    recs.sort(key=lambda r: r["index"])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_batch.json")
    with open(out, "w") as f:
        json.dump({"config": "C3 512 instances, n log-uniform [500, 50000], q in 20..64",
                   "frac": 0.125, "alpha": 2.0, "instances": recs}, f, indent=0)
    print(out, sum(r["n_colors"] for r in recs), flush=True)


_SLICE = {}


def _count_slice(bounds):
    g = _SLICE
    cnt, tests = oracle.count_conflict_edges(g["chars"], g["ids"], g["lists"], g["P"], g["rel"], *bounds)
    return cnt, tests


def c4_main(workers):
    """Colours of the n = 2M workload (seed 0) and every iteration's sizes."""
    import multiprocessing as mp

    cfg = wl.C4
    oracle.build(force=False)
    x, z = wl.make(cfg)
    seed = 0
    t = time.time()
    nc, col, st = oracle.color_classes(x, z, cfg.q, seed, cfg.frac, cfg.alpha, cfg.relation, count_edges=False)
    t_color = time.time() - t
    print(f"C4 colours: {nc} in {t_color:.0f} s, {len(st)} iterations", flush=True)
    chars = oracle.decode(x, z, cfg.q)
    t = time.time()
    ctx = mp.get_context("fork")
    for k, it in enumerate(st):
        ell = k + 1
        # iteration ell's vertex set: the vertices not coloured before it,
        # i.e. whose colour id is at or above its palette offset
        ids = np.nonzero(col >= it["offset"])[0].astype(np.int32)
        assert ids.shape[0] == it["m"]
        lists = oracle.sample_lists(seed, ell, ids, it["P"], it["T"])
        _SLICE.update(chars=chars, ids=ids, lists=lists, P=it["P"], rel=cfg.relation)
        nsl = max(1, min(8 * workers, it["P"]))
        cuts = [it["P"] * j // nsl for j in range(nsl + 1)]
        with ctx.Pool(workers) as pool:
            parts = pool.map(_count_slice, list(zip(cuts[:-1], cuts[1:])))
        it["edges"] = int(sum(c for c, _ in parts))
        assert sum(tt for _, tt in parts) == it["pair_tests"]
        print(f"  iteration {ell}: m={it['m']} edges={it['edges']} ({time.time() - t:.0f} s)", flush=True)
    rec = {
        "config": cfg.name,
        "n": cfg.n,
        "q": cfg.q,
        "probs": list(cfg.probs),
        "gen_seed": cfg.seed,
        "seed": seed,
        "frac": cfg.frac,
        "alpha": cfg.alpha,
        "relation": cfg.relation,
        "n_colors": nc,
        "colors_sha256": hashlib.sha256(np.ascontiguousarray(col, dtype="<i4").tobytes()).hexdigest(),
        "colors_head": col[:32].tolist(),
        "iters": st,
        "oracle_seconds": round(t_color, 1),
        "edge_count_seconds": round(time.time() - t, 1),
        "method": "edge-free oracle colouring (colour classes); edges counted per colour slice",
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_seed0.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(out, nc, flush=True)


def c2_dynamic_main(divisor):
    """C2, seed 0, coloured by the round form of Alg. 2 (the stored result)
    and by the sequential Alg. 2 and the static order (colour counts)."""
    cfg = wl.C2
    oracle.build(force=False)
    x, z = wl.make(cfg)
    seed = 0
    t = time.time()
    nc, col, st = oracle.color(x, z, cfg.q, seed, cfg.frac, cfg.alpha, cfg.relation, dynamic=True,
                               rounds_divisor=divisor)
    secs = round(time.time() - t, 1)
    print(f"C2 round form (divisor {divisor}): {nc} colours in {secs} s", flush=True)
    nseq, _, stseq = oracle.color(x, z, cfg.q, seed, cfg.frac, cfg.alpha, cfg.relation, dynamic=True)
    print(f"C2 sequential Alg. 2: {nseq} colours", flush=True)
    nst, _, _ = oracle.color(x, z, cfg.q, seed, cfg.frac, cfg.alpha, cfg.relation)
    rec = {
        "config": cfg.name, "n": cfg.n, "q": cfg.q, "probs": list(cfg.probs), "gen_seed": cfg.seed, "seed": seed,
        "frac": cfg.frac, "alpha": cfg.alpha, "relation": cfg.relation, "colourer": "dynamic rounds",
        "divisor": divisor, "n_colors": nc,
        "colors_sha256": hashlib.sha256(np.ascontiguousarray(col, dtype="<i4").tobytes()).hexdigest(),
        "colors_head": col[:32].tolist(), "iters": st, "oracle_seconds": secs,
        "n_colors_sequential_alg2": nseq, "iterations_sequential_alg2": len(stseq), "n_colors_static": nst,
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_dynamic_seed0.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(out, nc, nseq, nst, flush=True)


def learned_main(beta):
    """Held-out instance 0 (n = 500,000, q = 96) coloured by Alg. 1 with each
    iteration's (f, alpha) from the FP64 twin of the stored network, given the
    iteration's features and beta.  Records the schedule and, per iteration,
    how far f m and alpha ln m sit from the integers P and T round to (a
    float32 evaluation of the network within 1e-4 relative of the FP64 one
    gives the same P and T when these margins are larger)."""
    import math

    pkg = os.path.join(ROOT, "paper_2401_06713_amd")
    params = np.load(os.path.join(pkg, "predictor.npy"))
    summary = json.load(open(os.path.join(pkg, "predictor.json")))
    if beta is None:
        beta = float(summary["acceptance_beta"])
    cfg = wl.LHELD0
    oracle.build(force=False)
    x, z = wl.make(cfg)
    seed = cfg.seed
    t = time.time()
    nc, col, st, sched = oracle.color_learned(x, z, cfg.q, seed, params.astype(np.float64), cfg.relation, beta)
    secs = round(time.time() - t, 1)
    margins = []
    for it, (f, a) in zip(st, sched):
        m = it["m"]
        fm, al = f * m, a * math.log(m) if m > 1 else 0.0

        def rel_gap(v):
            return abs(v - round(v)) / max(abs(v), 1e-300)

        margins.append({"fm": fm, "fm_rel_gap": rel_gap(fm), "alpha_ln_m": al, "alpha_ln_m_rel_gap": rel_gap(al)})
    rec = {
        "config": cfg.name, "n": cfg.n, "q": cfg.q, "probs": list(cfg.probs), "gen_seed": cfg.seed, "seed": seed,
        "relation": cfg.relation, "beta": beta,
        "predictor_sha256": hashlib.sha256(open(os.path.join(pkg, "predictor.npy"), "rb").read()).hexdigest(),
        "n_colors": nc,
        "colors_sha256": hashlib.sha256(np.ascontiguousarray(col, dtype="<i4").tobytes()).hexdigest(),
        "colors_head": col[:32].tolist(), "iters": st, "schedule": sched.tolist(), "rounding_margins": margins,
        "oracle_seconds": secs,
        "method": "Alg. 1 with the FP64 network twin choosing (f, alpha) per iteration; edge-free colouring "
                  "(colour classes), edges counted",
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "l_learned_seed7000000.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(out, nc, secs, flush=True)


def main():
    name = sys.argv[1]
    if name == "Llearned":
        return learned_main(float(sys.argv[2]) if len(sys.argv) > 2 else None)
    if name == "C2dyn":
        return c2_dynamic_main(int(sys.argv[2]) if len(sys.argv) > 2 else 16)
    if name == "C3":
        return batch_main(int(sys.argv[2]) if len(sys.argv) > 2 else 6)
    if name == "C4":
        return c4_main(int(sys.argv[2]) if len(sys.argv) > 2 else 6)
    seeds = [int(s) for s in sys.argv[2:]] or [0]
    cfg = CONFIGS[name]
    oracle.build(force=False)
    x, z = wl.make(cfg)
    for seed in seeds:
        t = time.time()
        nc, col, st = oracle.color(x, z, cfg.q, seed, cfg.frac, cfg.alpha, cfg.relation)
        rec = {
            "config": cfg.name,
            "n": cfg.n,
            "q": cfg.q,
            "probs": list(cfg.probs),
            "gen_seed": cfg.seed,
            "seed": seed,
            "frac": cfg.frac,
            "alpha": cfg.alpha,
            "relation": cfg.relation,
            "n_colors": nc,
            "colors_sha256": hashlib.sha256(np.ascontiguousarray(col, dtype="<i4").tobytes()).hexdigest(),
            "colors_head": col[:32].tolist(),
            "iters": st,
            "oracle_seconds": round(time.time() - t, 1),
        }
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name.lower()}_seed{seed}.json")
        with open(out, "w") as f:
            json.dump(rec, f, indent=1)
        print(out, nc, rec["oracle_seconds"], flush=True)


if __name__ == "__main__":
    main()
