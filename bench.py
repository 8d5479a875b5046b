"""Benchmark: one step = one full palette colouring (every iteration of
Alg. 1: lists, buckets, pair count + fill, list colouring, compaction) of a
synthetic Pauli-string workload, with the strings already resident in HBM.

Prints ONE JSON line (rank 0).  `value` is pair tests per second of
end-to-end step time; the line also carries conflict edges per second,
end-to-end seconds, the colour count, the roofline of the dominant kernel
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-tests/s + end-to-end s and #colours, learned vs fixed params, 1 GPU"
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # INT32 lanes per clock x clock: 39.3 Tops/s
MFMA_I8_PEAK_TOPS = 5000.0  # dense int8 MFMA, 5.0 POP/s
HBM_PEAK_GBS = 8000.0


# HBM bytes of the pair kernel's and the CSR fill's iteration-1 launches on
# the default workload, from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE;
# summary and commands in profiles/pair_and_fill_c4_n2000000_q128_counters.md),
# each scaled by what the counter read for a 1 GiB device copy in the same
# runs.  Valid only for the kernel source they were taken from (its SHA-256).
PAIR_TRAFFIC = {
    "workload": "C4 n=2000000 q=128 pI=0.8",
    "path": "valu",
    "source": "paper_2401_06713_amd/csrc/relate.hip",
    "sha256": "a4eb31278c6673bdf4a234cbcec3ec625b313a2efa81133f8732b8622a2ac835",
    "fetch_kib": 1337859.8,
    "fetch_scale": 1048576.0 / 524315.6,
    "write_kib": 2874454.8,
    "write_scale": 1048576.0 / 1048576.0,
}

FILL_TRAFFIC = {
    "workload": "C4 n=2000000 q=128 pI=0.8",
    "path": "valu",
    "source": "paper_2401_06713_amd/csrc/pairs.hip",
    "sha256": "d0553654c5e9c530158633d308c49bdc762ae6b5a59446278cc46b674ce8251f",
    "fetch_kib": 5705837.75,
    "fetch_scale": 1048576.0 / 524315.6,
    "write_kib": 29703929.0,
    "write_scale": 1048576.0 / 1048576.0,
}


def recorded_traffic(workload: str, path: str, rec):
    import hashlib

    if rec is None or workload != rec["workload"] or path != rec["path"]:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
            return None  # the kernel changed since the counters were taken
    return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info() -> dict:
    """The host the CPU baseline ran on: CPU model, logical CPUs, memory."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    ram = round(int(line.split()[1]) / 2**20, 1)  # GiB
                    break
    except OSError:
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count(), "ram_gib": ram}


def cpu_baseline(cfg, x, z, budget_s: float):
    """The oracle's conflict-graph build on a slice of iteration 1's colour
    buckets (single thread), scaled to pair tests per second."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    ch = oracle.decode(x, z, cfg.q)
    ids = np.arange(cfg.n, dtype=np.int32)
    P, T = oracle.params(cfg.n, cfg.frac, cfg.alpha)
    lists = oracle.sample_lists(0, 1, ids, P, T)
    # calibrate on a small slice, then size the timed slice to the budget
    probe = max(1, P // 200)
    t = time.perf_counter()
    _, _, tests = oracle.conflict_edges_bucketed(ch, ids, lists, P, cfg.relation, 0, probe, want_edges=False)
    rate = tests / max(time.perf_counter() - t, 1e-6)
    want = int(budget_s * rate)
    per_colour = max(tests / probe, 1.0)
    hi = int(min(P, max(probe, want / per_colour)))
    t = time.perf_counter()
    _, edges, tests = oracle.conflict_edges_bucketed(ch, ids, lists, P, cfg.relation, 0, hi, want_edges=False)
    dt = time.perf_counter() - t
    return {
        "value": tests / dt,
        "unit": "pair-tests/s",
        "cores": 1,
        "host": host_info(),
        "kind": "oracle",
        "sample": f"{cfg.name}: iteration-1 conflict build over colour buckets [0,{hi}) of {P} "
                  f"({tests} pair tests, {edges} edges, {dt:.1f} s, single-threaded C oracle)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C4", choices=["C1", "C2", "C3", "C4"])
    ap.add_argument("--path", default="valu", choices=["auto", "valu", "mfma"],
                    help="pair pass: popcount tile kernel (valu), int8 MFMA kernel with popcount for buckets "
                         "above its LDS cap (mfma), or the library's choice (auto)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-fixed comparison")
    ap.add_argument("--beta", type=float, default=None,
                    help="trade-off input of the learned parameters (weight of the colour count); default: the "
                         "beta the stored network's held-out evaluation accepted")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy MIB MiB device to device once (a plain copy of known size "
                         "that calibrates the HBM byte counters of a profiler run)")
    ap.add_argument("--tune", action="store_true",
                    help="run the launch-shape tuner first (its colourings run before the warm-up)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the method runs on a single device); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs as a single process", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2401_06713_amd as pk
    from paper_2401_06713_amd import learn, tune
    from paper_2401_06713_amd import workloads as wl

    torch.cuda.set_device(0)
    batch = args.config == "C3"
    if batch:
        cfgs = wl.batch_instances()
        log(f"bench: generating {len(cfgs)} batch instances")
        insts = [wl.make(c) for c in cfgs]
        h = pk.PicassoBatch([(x, z, c.q) for (x, z), c in zip(insts, cfgs)])
        out = torch.empty(h.n, dtype=torch.int32, device="cuda")
        run_args = ([c.seed for c in cfgs], [c.frac for c in cfgs], [c.alpha for c in cfgs],
                    [c.relation for c in cfgs])

        def step():
            return int(h.color_batch_device(out, *run_args).sum())

        cfg = max(cfgs, key=lambda c: c.n)  # the CPU baseline's sample instance
        x, z = insts[cfgs.index(cfg)]
        workload = {"workload": f"C3 batch of {len(cfgs)} instances, n log-uniform [500, 50000], q in 20..64, "
                                "pI in [0.5, 0.85], anticommute or QWC per instance",
                    "instances": len(cfgs), "total_strings": h.n, "palette_frac": 0.125, "list_size_alpha": 2.0}
    else:
        cfg = {"C1": wl.C1, "C2": wl.C2, "C4": wl.C4}[args.config]
        log(f"bench: generating {cfg.name}")
        x, z = wl.make(cfg)
        xd = torch.from_numpy(x.view(np.int64)).cuda()
        zd = torch.from_numpy(z.view(np.int64)).cuda()
        out = torch.empty(cfg.n, dtype=torch.int32, device="cuda")
        h = pk.Picasso(xd, zd, cfg.q)
        run_args = (args.seed, cfg.frac, cfg.alpha, cfg.relation)

        def step():
            return h.color_device(out, *run_args)

        workload = {"workload": cfg.name, "n": cfg.n, "q": cfg.q, "probs": list(cfg.probs), "seed": args.seed,
                    "palette_frac": cfg.frac, "list_size_alpha": cfg.alpha,
                    "relation": ["anticommute", "qwc"][cfg.relation]}
    tuned = None
    if args.tune:
        if batch:
            tuned = tune.tune(h, *run_args, use_cache=False, log=log)
        else:
            tuned = tune.tune(h, [args.seed], [cfg.frac], [cfg.alpha], [cfg.relation], use_cache=False, log=log)
        log(f"bench: tuned {tuned}")
    else:
        h.set_option(pk.OPT_PAIR_PATH, {"auto": 0, "valu": 1, "mfma": 2}[args.path])
    h.set_option(pk.OPT_TIMING, 1)

    for i in range(args.warmup):
        nc = step()
        log(f"bench: warmup {i + 1}/{args.warmup}: {nc} colours")
    torch.cuda.synchronize()
    per_step = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        nc = step()
        per_step.append(h.stats())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"bench: {args.steps} steps in {elapsed:.3f} s")
    st = per_step[-1]
    ms_step = elapsed * 1e3 / args.steps
    pair_tests = st["pair_tests"]
    edges = st["edges"]

    # dominant kernel: the pair pass (every pair test), timed with HIP events
    # on the library's stream around its launches.  The roofline is taken on
    # its iteration-1 launch (the bulk of the pair tests; later iterations'
    # launches are small enough that launch latency dominates them).
    count_ms = sum(it["ms_count"] for s in per_step for it in s["iters"])
    fill_ms = sum(it["ms_fill"] for s in per_step for it in s["iters"])
    color_ms = sum(it["ms_color"] for s in per_step for it in s["iters"])
    launches = sum(len(s["iters"]) for s in per_step)
    first = [s["iters"][0] for s in per_step]
    ms1 = sum(it["ms_count"] for it in first) / len(first)
    tests1 = first[0]["pair_tests"]
    W = (h.q + 63) // 64
    ops_per_test = 8 * W + 1  # per 32-bit half of a word: 2 AND + 1 XOR; 2W-1 XOR merges, popcount, AND
    mfma = first[0]["pair_path"] == pk.PATH_MFMA
    if mfma:
        ops1 = 2 * (2 * h.q) * tests1  # a dot product of 2q bytes per pair (largest q of a batch)
        peak, unit, bound = MFMA_I8_PEAK_TOPS, "TOPS", "mfma"
        ops_all = sum(2 * (2 * h.q) * s["pair_tests"] for s in per_step)
    else:
        ops1 = ops_per_test * tests1
        peak, unit, bound = VALU_PEAK_TOPS, "Tops/s", "alu"
        ops_all = sum(ops_per_test * s["pair_tests"] for s in per_step)
    achieved = ops1 / (ms1 * 1e-3) / 1e12
    traffic = recorded_traffic(workload["workload"], args.path, PAIR_TRAFFIC) if not batch else None
    roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": traffic,
            "kernel": "pair pass (relation bit matrices), iteration-1 launch",
            "avg_launch_ms": ms1, "pair_tests_per_launch": tests1, "ops_per_pair_test": ops1 / tests1,
            "all_launches": {"launches": launches, "avg_launch_ms": count_ms / max(launches, 1),
                             "frac": ops_all / (count_ms * 1e-3) / 1e12 / peak}}
    if traffic:
        roof["traffic_unit"] = "bytes per launch (HBM, counter-scaled)"

    # edge compaction (CSR fill), bound by HBM: it writes two int32 column
    # indices per undirected conflict edge; reading the bucket relation rows
    # and member ids is overhead of this design, not counted
    fill1 = sum(it["ms_fill"] for it in first) / len(first)
    edges1 = first[0]["edges"]
    fill_bytes = 8 * edges1
    fill_gbs = fill_bytes / (fill1 * 1e-3) / 1e9 if fill1 > 0 else None
    fill = {"bound": "hbm", "kernel": "CSR fill (edge compaction), iteration-1 launch", "avg_launch_ms": fill1,
            "edges_per_launch": edges1, "algorithmic_bytes": fill_bytes, "achieved": fill_gbs,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fill_gbs / HBM_PEAK_GBS if fill_gbs else None,
            "traffic": None}
    ftraffic = recorded_traffic(workload["workload"], args.path, FILL_TRAFFIC) if not batch else None
    if ftraffic and fill1 > 0:
        fill["traffic"] = ftraffic
        fill["traffic_GBs"] = ftraffic / (fill1 * 1e-3) / 1e9
        fill["traffic_unit"] = "bytes per launch (HBM, counter-scaled)"
    graph_ms = sum(it["ms_graph"] for s in per_step for it in s["iters"]) / args.steps

    # colour counts over colouring seeds 0-4 (untimed)
    seeds_nc = None
    dyn = None
    if not batch:
        seeds_nc = [int(h.color_device(out, sd, cfg.frac, cfg.alpha, cfg.relation)) for sd in range(5)]
        # the dynamic-order colourer (Alg. 2 in rounds) on the same workload:
        # colours and end-to-end time beside the static order's
        h.set_option(pk.OPT_COLOURER, pk.COLOURER_DYNAMIC)
        h.color_device(out, *run_args)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ncd = int(h.color_device(out, *run_args))
        torch.cuda.synchronize()
        sd_ = h.stats()
        dyn = {"n_colors": ncd, "ms": (time.perf_counter() - t1) * 1e3, "iterations": sd_["n_iters"],
               "rounds": sum(it["jp_rounds"] for it in sd_["iters"]), "divisor": 16,
               "ms_color": sum(it["ms_color"] for it in sd_["iters"])}
        h.set_option(pk.OPT_COLOURER, pk.COLOURER_STATIC)

    workload["pair_path"] = args.path
    if tuned:
        workload["tuned"] = {k: tuned[k] for k in ("cap", "jp_batch", "graph")}
    line = {
        "metric": METRIC,
        "value": pair_tests / (ms_step * 1e-3),
        "unit": "pair-tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "median_call_ms": sorted(s["ms_total"] for s in per_step)[len(per_step) // 2],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": workload,
        "end_to_end_s": ms_step * 1e-3,
        "n_colors": nc,
        "iterations": st["n_iters"],
        "pair_tests": pair_tests,
        "conflict_edges": edges,
        "conflict_edges_per_s": edges / (ms_step * 1e-3),
        "conflict_edges_per_s_graph_build": edges / (graph_ms * 1e-3) if graph_ms > 0 else None,
        "phase_ms_per_step": {"graph_build": graph_ms, "pair_pass": count_ms / args.steps,
                              "pair_fill": fill_ms / args.steps, "list_color": color_ms / args.steps},
        "peak_device_bytes": st["peak_device_bytes"],
        "roofline": roof,
        "edge_compaction": fill,
    }
    if seeds_nc:
        line["n_colors_seeds_0_4"] = {"n_colors": seeds_nc, "mean": sum(seeds_nc) / len(seeds_nc)}
    if dyn:
        line["dynamic_colourer"] = dyn
    h.close()
    params = np.load(learn.PREDICTOR) if os.path.exists(learn.PREDICTOR) else None
    if params is not None and params.shape != (pk.MLP_NPARAMS,):
        params = None  # stored for another network shape
    if not batch and not args.no_learned and params is not None:
        # learned parameters (the stored network) against the fixed ones, each
        # on a fresh handle so that peak device bytes count only its own run
        log("bench: learned vs fixed parameters")
        mlp = pk.Mlp(params)
        summary_path = os.path.splitext(learn.PREDICTOR)[0] + ".json"
        summary = json.load(open(summary_path)) if os.path.exists(summary_path) else {}
        beta = args.beta if args.beta is not None else (summary.get("acceptance_beta") or 0.3)
        cmp = {"beta": beta}
        for name in ("fixed", "fixed_tail", "learned"):
            hh = pk.Picasso(xd, zd, cfg.q)
            hh.set_option(pk.OPT_PAIR_PATH, pk.PATH_VALU)
            # the learned run consults the network every iteration, so it
            # cannot hand the last iterations to the tail kernel: the fixed
            # run is timed both ways
            hh.set_option(pk.OPT_TAIL, int(name == "fixed_tail"))
            run = (lambda: hh.color(args.seed, cfg.frac, cfg.alpha, cfg.relation)[0]) if name != "learned" else \
                (lambda: hh.color_learned(mlp, args.seed, cfg.relation, beta)[0])
            run()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(3):
                ncl = run()
            ms_l = (time.perf_counter() - t1) * 1e3 / 3
            sl = hh.stats()
            cmp[name] = {"n_colors": ncl, "ms": ms_l, "max_edges": sl["max_edges"],
                         "peak_device_bytes": sl["peak_device_bytes"], "iterations": sl["n_iters"]}
            if name == "learned":
                cmp[name]["first_iteration_params"] = [sl["iters"][0]["P"], sl["iters"][0]["T"]]
            hh.close()
        mlp.close()
        cmp["note"] = "host-output calls; network trained on sweeps over %s instances, n in %s" % (
            summary.get("train_instances"), summary.get("n_range"))
        line["learned_vs_fixed"] = cmp
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = args.copy_calibration << 20
        del src, dst
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(cfg, x, z, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
