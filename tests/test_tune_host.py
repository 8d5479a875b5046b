"""Host-side parts of the launch-shape tuner that need no GPU: the workload
signature its cache is keyed by, and the cache file's round trip."""
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
