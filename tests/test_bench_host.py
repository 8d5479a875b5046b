"""Host-side parts of bench.py that run without a GPU: the single-GPU guard,
the gating of recorded counter traffic on the kernel source it was taken
from, and the CPU-baseline leg (the oracle timed on a bounded sample)."""
import hashlib
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2401_06713_amd import workloads as wl  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_recorded_traffic_is_gated_on_workload_and_source():
    for recorded in (bench.PAIR_TRAFFIC, bench.FILL_TRAFFIC):
        with open(os.path.join(ROOT, recorded["source"]), "rb") as f:
            current = hashlib.sha256(f.read()).hexdigest()
        rec = dict(recorded, sha256=current)
        got = bench.recorded_traffic(rec["workload"], rec["path"], rec)
        want = (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0
        assert got == want and got > 0
        other = "C2 n=200000 q=48 pI=0.7" if rec["workload"].startswith("C4") else "C4 n=2000000 q=128 pI=0.8"
        assert bench.recorded_traffic(other, rec["path"], rec) is None
        assert bench.recorded_traffic(rec["workload"], "mfma", rec) is None
        stale = dict(rec, sha256="0" * 64)  # the kernel source changed since the counters were taken
        assert bench.recorded_traffic(rec["workload"], rec["path"], stale) is None
    assert bench.recorded_traffic("C2 n=200000 q=48 pI=0.7", "valu", None) is None


def test_cpu_baseline_leg_on_a_small_sample():
    cfg = wl.C1
    x, z = wl.make(cfg)
    out = bench.cpu_baseline(cfg, x, z, budget_s=0.3)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "pair-tests/s"
    assert np.isfinite(out["value"]) and out["value"] > 0
    assert cfg.name in out["sample"]
    assert set(out["host"]) == {"cpu", "logical_cpus", "ram_gib"} and out["host"]["logical_cpus"] >= 1
