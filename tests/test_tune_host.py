"""Host-side parts of the launch-shape tuner that need no GPU: the workload
signature its cache is keyed by, the cache file's round trip, and how a
configuration maps to handle options."""
from paper_2401_06713_amd import tune


class FakeHandle:
    def __init__(self, W, n, count=1):
        self.W, self.n, self.count = W, n, count


def test_signature_classes():
    assert tune.signature(FakeHandle(1, 200_000), [0]) == "W1-rel0-n2^18-nb2^0"
    # relations are a set, sizes a power-of-two class
    assert tune.signature(FakeHandle(2, 2_000_000, 512), [1, 0, 1]) == "W2-rel01-n2^21-nb2^9"
    assert tune.signature(FakeHandle(1, 200_000), [0]) == tune.signature(FakeHandle(1, 300_000), [0])
    assert tune.signature(FakeHandle(1, 200_000), [2]) != tune.signature(FakeHandle(1, 200_000), [0])


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(path) == {}
    entry = {"cap": 64, "jp_batch": 32, "graph": 1, "ms": 13.9, "default_ms": 14.6}
    tune.save_cache({"W1-rel0-n2^18-nb2^0": entry}, path)
    assert tune.load_cache(path) == {"W1-rel0-n2^18-nb2^0": entry}
    with open(path, "w") as f:
        f.write("{not json")
    assert tune.load_cache(path) == {}  # a damaged cache is ignored, not fatal


class OptionRecorder:
    def __init__(self):
        self.opts = {}

    def set_option(self, key, value):
        self.opts[key] = value


def test_apply_maps_caps_to_paths():
    import paper_2401_06713_amd as pk

    # the tuner starts from the library's default: every bucket on the popcount kernel
    assert tune.DEFAULT["cap"] == 0
    h = OptionRecorder()
    tune.apply(h, dict(tune.DEFAULT))
    assert h.opts[pk.OPT_PAIR_PATH] == pk.PATH_VALU and h.opts[pk.OPT_MFMA_CAP] == -1
    # a positive cap: buckets up to it on the MFMA kernel
    tune.apply(h, {"cap": 64, "jp_batch": 16, "graph": 0})
    assert h.opts[pk.OPT_PAIR_PATH] == pk.PATH_MFMA and h.opts[pk.OPT_MFMA_CAP] == 64
    assert h.opts[pk.OPT_JP_BATCH] == 16 and h.opts[pk.OPT_GRAPH] == 0
    # cap -1: every bucket the MFMA kernel holds (never the library's auto)
    tune.apply(h, {"cap": -1, "jp_batch": 32, "graph": 1})
    assert h.opts[pk.OPT_PAIR_PATH] == pk.PATH_MFMA and h.opts[pk.OPT_MFMA_CAP] == -1
    assert -1 in tune.CAPS and 0 in tune.CAPS
