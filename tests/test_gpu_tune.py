"""The launch-shape tuner: every configuration it tries colours identically
(it checks that itself), the configuration it picks still matches the
oracle, and its cache round-trips."""
import json
import sys

import numpy as np
import pytest

import paper_2401_06713_amd as pk
from paper_2401_06713_amd import tune

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_batch import mixed_instances  # noqa: E402

pytestmark = pytest.mark.gpu


def test_tuner_picks_valid_config_and_caches(orc, tmp_path):
    insts = [d for d in mixed_instances(14, 9) if d["x"].shape[0] > 0]
    args = ([d["seed"] for d in insts], [d["frac"] for d in insts], [d["alpha"] for d in insts],
            [d["rel"] for d in insts])
    cache = str(tmp_path / "tune.json")
    with pk.PicassoBatch([(d["x"], d["z"], d["q"]) for d in insts]) as h:
        got = tune.tune(h, *args, repeats=1, sweeps=1, cache_file=cache, log=print)
        assert not got["cached"] and got["ms"] <= got["default_ms"]
        nc, cols = h.color_batch(*args)
    for i, d in enumerate(insts):
        rnc, rcol, _ = orc.color(d["x"], d["z"], d["q"], d["seed"], d["frac"], d["alpha"], d["rel"])
        assert nc[i] == rnc and np.array_equal(cols[i], rcol)
    stored = json.load(open(cache))
    assert got["key"] in stored
    with pk.PicassoBatch([(d["x"], d["z"], d["q"]) for d in insts]) as h2:
        again = tune.tune(h2, *args, cache_file=cache)
        assert again["cached"] and {k: again[k] for k in ("cap", "jp_batch", "graph")} == \
            {k: got[k] for k in ("cap", "jp_batch", "graph")}
