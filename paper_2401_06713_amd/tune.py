"""Autotuner for the colouring's launch shapes.

The knobs, all plain options of a handle:

* pair tile shape: buckets of at most `cap` members take the int8 MFMA
  kernel (32 x 32 output tiles over a bucket staged whole in LDS), larger
  ones the popcount kernel (64-row tiles, one wave per row tile);
  `cap = 0` sends every bucket to the popcount kernel (the default) and
  `cap = -1` every bucket the MFMA kernel's LDS rows can hold;
* colouring rounds launched between two host progress checks;
* whether a full batch of rounds is replayed from a captured HIP graph.

The tuner times whole colourings of the caller's own workload (wall time
of the library call, best of `repeats`), walks the knobs one at a time from
the defaults (coordinate descent, two sweeps), and caches the winner per
workload signature (string words, relations, size class, instance count) in
a JSON file, so later handles of the same shape start tuned.  Every
candidate produces the same colouring: a knob changes launch shapes, never
results; the tuner checks that as it goes.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

import paper_2401_06713_amd as pk

CACHE_ENV = "PICASSO_TUNE_CACHE"
DEFAULT = {"cap": 0, "jp_batch": 32, "graph": 1}
CAPS = (0, 32, 64, 128, 256, -1)
JP_BATCHES = (4, 8, 16, 32, 64)
GRAPHS = (0, 1)


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "picasso_tune.json")


def signature(h: pk.Picasso, relations) -> str:
    rels = sorted(set(int(r) for r in np.atleast_1d(relations)))
    nb = getattr(h, "count", 1)
    return f"W{h.W}-rel{''.join(map(str, rels))}-n2^{round(math.log2(max(h.n, 1)))}-nb2^{round(math.log2(max(nb, 1)))}"


def apply(h: pk.Picasso, cfg: dict):
    """Set a tuned configuration on a handle."""
    cap = int(cfg["cap"])
    h.set_option(pk.OPT_PAIR_PATH, pk.PATH_VALU if cap == 0 else pk.PATH_MFMA)
    h.set_option(pk.OPT_MFMA_CAP, cap if cap > 0 else -1)
    h.set_option(pk.OPT_JP_BATCH, int(cfg["jp_batch"]))
    h.set_option(pk.OPT_GRAPH, int(cfg["graph"]))


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str | None = None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _runner(h, seeds, fracs, alphas, relations):
    """A function running one whole colouring; returns (ms, fingerprint)."""
    if isinstance(h, pk.PicassoBatch):
        def run():
            t = time.perf_counter()
            nc, cols = h.color_batch(seeds, fracs, alphas, relations)
            ms = (time.perf_counter() - t) * 1e3
            return ms, (tuple(nc.tolist()), hash(np.concatenate(cols).tobytes()) if cols else 0)
    else:
        seed, frac, alpha, rel = (np.atleast_1d(v)[0] for v in (seeds, fracs, alphas, relations))

        def run():
            t = time.perf_counter()
            nc, col = h.color(int(seed), float(frac), float(alpha), int(rel))
            ms = (time.perf_counter() - t) * 1e3
            return ms, (nc, hash(col.tobytes()))
    return run


def tune(h: pk.Picasso, seeds, fracs, alphas, relations, repeats: int = 2, sweeps: int = 2, use_cache: bool = True,
         cache_file: str | None = None, log=None) -> dict:
    """Tune the handle's knobs on its own workload; returns the chosen
    configuration (also applied to the handle) with its timing."""
    key = signature(h, relations)
    cache = load_cache(cache_file) if use_cache else {}
    if use_cache and key in cache:
        apply(h, cache[key])
        return dict(cache[key], cached=True, key=key)
    run = _runner(h, seeds, fracs, alphas, relations)
    apply(h, DEFAULT)
    run()  # warm-up: allocations reach their working size
    timings = {}
    reference = None

    def measure(cfg):
        nonlocal reference
        k = (cfg["cap"], cfg["jp_batch"], cfg["graph"])
        if k in timings:
            return timings[k]
        try:
            apply(h, cfg)
            best = math.inf
            for _ in range(repeats):
                ms, fp = run()
                if reference is None:
                    reference = fp
                elif fp != reference:
                    raise RuntimeError(f"tuning candidate {cfg} changed the colouring")
                best = min(best, ms)
        except pk.PicassoError as e:
            if e.code != pk.EINVAL:
                raise
            best = math.inf  # not available for this q / relation
        timings[k] = best
        if log:
            log(f"tune {key}: {cfg} -> {best:.2f} ms")
        return best

    cur = dict(DEFAULT)
    best_ms = measure(cur)
    for _ in range(sweeps):
        changed = False
        for knob, values in (("cap", CAPS), ("jp_batch", JP_BATCHES), ("graph", GRAPHS)):
            for v in values:
                cand = dict(cur, **{knob: v})
                ms = measure(cand)
                if ms < best_ms:
                    best_ms, cur, changed = ms, cand, True
        if not changed:
            break
    apply(h, cur)
    result = dict(cur, ms=best_ms, default_ms=timings[(DEFAULT["cap"], DEFAULT["jp_batch"], DEFAULT["graph"])])
    if use_cache:
        cache = load_cache(cache_file)
        cache[key] = result
        save_cache(cache, cache_file)
    return dict(result, cached=False, key=key)
