"""Write stored oracle results for the full-size single-instance workloads.

Calls only the CPU oracle (oracle/) and the seeded input generator; the
HIP path is never involved.  Each JSON file holds the colour count, the
SHA-256 of the little-endian int32 colour array and the per-iteration sizes.

    python tests/golden/make_golden.py C2 [seed ...]
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

CONFIGS = {"C1": wl.C1, "C2": wl.C2, "C4": wl.C4}


def main():
    name = sys.argv[1]
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
