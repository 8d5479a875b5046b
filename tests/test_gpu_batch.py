"""Batched colouring vs the CPU oracle, instance by instance.

A batch handle colours every instance as a single-instance call would
colour it alone, so each instance's colours must equal the oracle's run
on that instance with that instance's arguments: bit-exact (integer
work).  The full 512-instance workload is checked against stored oracle
results (tests/golden/c3_batch.json, written by make_golden.py from the
oracle alone).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import paper_2401_06713_amd as pk
from paper_2401_06713_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_batch.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_instances(count, seed):
    """Uneven instances: sizes 0..1500, q across one to four words, all three
    relations, per-instance seeds, palette fractions and list multipliers."""
    rng = np.random.default_rng(seed)
    sizes = [0, 1, 2, 3, 17] + [int(v) for v in np.exp(rng.uniform(np.log(20), np.log(1500), count - 5))]
    qs = rng.choice([1, 7, 20, 48, 64, 65, 100, 130, 200], count)
    out = []
    for i in range(count):
        n, q = sizes[i], int(qs[i])
        pI = float(rng.uniform(0.3, 0.85))
        r = (1 - pI) / 3
        maxn = 4 ** q - 1 if q < 8 else n
        n = min(n, maxn)
        x, z = wl.pauli_strings(n, q, (pI, r, r, r), seed=1000 + i) if n else (
            np.zeros((0, (q + 63) // 64), np.uint64), np.zeros((0, (q + 63) // 64), np.uint64))
        out.append(dict(x=x, z=z, q=q, seed=int(rng.integers(0, 2**63)), frac=float(rng.choice([0.08, 0.125, 0.3])),
                        alpha=float(rng.choice([1.0, 2.0, 3.0])), rel=int(rng.integers(0, 3))))
    rng.shuffle(out)
    return out


def color_batch(insts, path=pk.PATH_AUTO, opts=()):
    with pk.PicassoBatch([(d["x"], d["z"], d["q"]) for d in insts]) as h:
        h.set_option(pk.OPT_PAIR_PATH, path)
        for k, v in opts:
            h.set_option(k, v)
        nc, cols = h.color_batch([d["seed"] for d in insts], [d["frac"] for d in insts],
                                 [d["alpha"] for d in insts], [d["rel"] for d in insts])
        return nc, cols, h.stats(), h.instance_stats()


@pytest.fixture(scope="module")
def mixed(orc):
    insts = mixed_instances(40, 7)
    refs = []
    for d in insts:
        if d["x"].shape[0] == 0:
            refs.append((0, np.zeros(0, np.int32), []))
        else:
            refs.append(orc.color(d["x"], d["z"], d["q"], d["seed"], d["frac"], d["alpha"], d["rel"]))
    return insts, refs


@pytest.mark.parametrize("path", [pk.PATH_VALU, pk.PATH_AUTO])
def test_batch_bit_exact_per_instance(mixed, path):
    insts, refs = mixed
    say("batch mixed", len(insts), "path", path)
    nc, cols, st, ist = color_batch(insts, path)
    for i, (d, (rnc, rcol, rst)) in enumerate(zip(insts, refs)):
        assert nc[i] == rnc, (i, d["q"], d["x"].shape[0])
        assert np.array_equal(cols[i], rcol), (i, d["q"], d["x"].shape[0])
        assert ist[i]["n_colors"] == rnc and ist[i]["n_iters"] == len(rst)
        assert ist[i]["n"] == d["x"].shape[0]
    assert st["n_colors"] == sum(r[0] for r in refs)
    assert st["n_iters"] == max(len(r[2]) for r in refs)


def test_batch_rounds_and_graph_options(mixed):
    """Plain launches, odd round counts, one round per check and either
    colour-bucket build give the same colouring as the defaults."""
    insts, refs = mixed
    for opts in (((pk.OPT_GRAPH, 0),), ((pk.OPT_JP_BATCH, 3),), ((pk.OPT_JP_BATCH, 1),),
                 ((pk.OPT_JP_BATCH, 64), (pk.OPT_GRAPH, 1)), ((pk.OPT_BUCKET_BUILD, 2),),
                 ((pk.OPT_BUCKET_BUILD, 1),)):
        say("batch options", opts)
        nc, cols, _, _ = color_batch(insts, pk.PATH_AUTO, opts)
        for i, (rnc, rcol, _) in enumerate(refs):
            assert nc[i] == rnc and np.array_equal(cols[i], rcol), (opts, i)


def test_batch_on_caller_stream_and_repeated_calls(mixed):
    """On a stream the caller owns (PICASSO_OPT_STREAM; the tail kernels run
    on the handle's second stream and are joined back to it), and on three
    calls in a row on one handle: the same colours and statistics."""
    import torch

    insts, refs = mixed
    s = torch.cuda.Stream()
    with pk.PicassoBatch([(d["x"], d["z"], d["q"]) for d in insts]) as h:
        args = ([d["seed"] for d in insts], [d["frac"] for d in insts], [d["alpha"] for d in insts],
                [d["rel"] for d in insts])
        h.set_option(pk.OPT_STREAM, s.cuda_stream)
        for rep in range(3):
            nc, cols = h.color_batch(*args)
            ist = h.instance_stats()
            for i, (rnc, rcol, rst) in enumerate(refs):
                assert nc[i] == rnc and np.array_equal(cols[i], rcol), (rep, i)
                assert ist[i]["n_iters"] == len(rst), (rep, i)
        h.set_option(pk.OPT_STREAM, 0)
    torch.cuda.synchronize()


def test_batch_equals_single_handles(mixed):
    insts, refs = mixed
    picked = [d for d in insts if d["x"].shape[0] > 0][:6]
    nc, cols, _, _ = color_batch(picked)
    for i, d in enumerate(picked):
        with pk.Picasso(d["x"], d["z"], d["q"]) as h:
            snc, scol = h.color(d["seed"], d["frac"], d["alpha"], d["rel"])
        assert snc == nc[i] and np.array_equal(scol, cols[i])


def test_batch_handle_rejects_single_instance_calls():
    insts = mixed_instances(6, 3)
    with pk.PicassoBatch([(d["x"], d["z"], d["q"]) for d in insts]) as h:
        for call in (lambda: h.color(0), lambda: h.sample_lists(0, 1, np.arange(2), 4, 2),
                     lambda: h.features(0, 1, np.arange(2), 0)):
            with pytest.raises(pk.PicassoError) as e:
                call()
            assert e.value.code == pk.EINVAL
    # a batch of one behaves as a single-instance handle
    d = [d for d in insts if d["x"].shape[0] > 3][0]
    with pk.PicassoBatch([(d["x"], d["z"], d["q"])]) as h:
        nc, col = h.color(d["seed"], d["frac"], d["alpha"], d["rel"])
        nc2, cols = h.color_batch([d["seed"]], [d["frac"]], [d["alpha"]], [d["rel"]])
    assert nc == nc2[0] and np.array_equal(col, cols[0])


def test_batch_all_empty():
    z0 = np.zeros((0, 1), np.uint64)
    with pk.PicassoBatch([(z0, z0, 5), (z0, z0, 70)]) as h:
        nc, cols = h.color_batch([1, 2], [0.1, 0.1], [2.0, 2.0], [0, 1])
    assert list(nc) == [0, 0] and all(c.size == 0 for c in cols)


def test_batch_invalid_arguments():
    x, z = wl.pauli_strings(10, 5, seed=1)
    bad = x.copy()
    bad[0, 0] |= np.uint64(1) << np.uint64(63)  # a bit above q
    with pytest.raises(pk.PicassoError) as e:
        pk.PicassoBatch([(x, z, 5), (bad, z, 5)])
    assert e.value.code == pk.EINVAL
    with pk.PicassoBatch([(x, z, 5), (x, z, 5)]) as h:
        with pytest.raises(pk.PicassoError):
            h.color_batch([0, 0], [0.1, 1.5], [2.0, 2.0], [0, 0])  # palette fraction above 1
        with pytest.raises(pk.PicassoError):
            h.color_batch([0, 0], [0.1, 0.1], [2.0, 2.0], [0, 3])  # unknown relation


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stored oracle results for the batch are not present")
def test_batch_c3_full_size_golden():
    """All 512 instances of the batched workload, bit-exact against the
    stored oracle colourings (count and SHA-256 of each colour array)."""
    gold = json.load(open(GOLDEN))["instances"]
    cfgs = wl.batch_instances()
    assert len(gold) == len(cfgs)
    say("generating", len(cfgs), "instances")
    insts = [wl.make(c) for c in cfgs]
    say("colouring")
    with pk.PicassoBatch([(x, z, c.q) for (x, z), c in zip(insts, cfgs)]) as h:
        nc, cols = h.color_batch([c.seed for c in cfgs], [c.frac for c in cfgs], [c.alpha for c in cfgs],
                                 [c.relation for c in cfgs])
        st = h.stats()
    say("batch", st["n_iters"], "iterations", round(st["ms_total"], 1), "ms")
    for i, (g, c) in enumerate(zip(gold, cfgs)):
        assert g["n"] == c.n and g["seed"] == c.seed and g["relation"] == c.relation
        assert nc[i] == g["n_colors"], i
        assert hashlib.sha256(np.ascontiguousarray(cols[i], dtype="<i4").tobytes()).hexdigest() == \
            g["colors_sha256"], i


def test_tail_kernel_matches_full_path(mixed):
    """Instances finished by the tail kernel (at most 256 vertices left) give
    the same colours and per-iteration sizes as the full path."""
    insts, refs = mixed
    nc_on, cols_on, st_on, ist_on = color_batch(insts, pk.PATH_AUTO, ((pk.OPT_TAIL, 1),))
    nc_off, cols_off, st_off, ist_off = color_batch(insts, pk.PATH_AUTO, ((pk.OPT_TAIL, 0),))
    assert np.array_equal(nc_on, nc_off)
    for a, b in zip(cols_on, cols_off):
        assert np.array_equal(a, b)
    assert ist_on == ist_off
    assert st_on["n_iters"] == st_off["n_iters"]
    for a, b in zip(st_on["iters"], st_off["iters"]):
        for k in ("m", "P", "T", "pair_tests", "edges", "colored"):
            assert a[k] == b[k], (k, a[k], b[k])
    assert any(it["pair_path"] == 0 for it in st_on["iters"])
