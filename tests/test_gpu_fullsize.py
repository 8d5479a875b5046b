"""Full-size workloads on the HIP path.

C2 (n=200,000, q=48): bit-exact against stored oracle results written by
tests/golden/make_golden.py (which calls only the CPU oracle), plus
properties that hold at any size: every colour class is independent in the
relation graph, colours lie in their iteration's palette, and each
iteration's sizes match.
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
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def class_pairs(col):
    """All pairs (a, b), a < b, of vertices with equal colours."""
    order = np.argsort(col, kind="stable")
    c = col[order]
    starts = np.flatnonzero(np.r_[True, c[1:] != c[:-1]])
    sizes = np.diff(np.r_[starts, len(c)])
    A, B = [], []
    for s in range(2, sizes.max(initial=1) + 1):
        st = starts[sizes == s]
        if st.size == 0:
            continue
        for i in range(s):
            for j in range(i + 1, s):
                A.append(order[st + i])
                B.append(order[st + j])
    if not A:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(A), np.concatenate(B)


def relation_np(x, z, a, b, rel):
    acc = np.zeros(a.shape[0], np.uint64)
    hit = np.zeros(a.shape[0], bool)
    par = np.zeros(a.shape[0], np.uint64)
    for w in range(x.shape[1]):
        t = (x[a, w] & z[b, w]) ^ (z[a, w] & x[b, w])
        par ^= t
        hit |= t != 0
    if rel == 0:
        return (np.bitwise_count(par) & 1).astype(bool)
    return hit


def check_valid(x, z, col, rel):
    a, b = class_pairs(col)
    assert not relation_np(x, z, a, b, rel).any()


@pytest.mark.parametrize("seed,path", [(0, pk.PATH_AUTO), (1, pk.PATH_AUTO), (2, pk.PATH_AUTO), (3, pk.PATH_AUTO),
                                       (4, pk.PATH_AUTO), (0, pk.PATH_VALU), (1, pk.PATH_MFMA)])
def test_c2_matches_oracle(seed, path):
    gpath = os.path.join(GOLDEN, f"c2_seed{seed}.json")
    if not os.path.exists(gpath):
        pytest.skip(f"no stored oracle result for seed {seed}")
    g = json.load(open(gpath))
    cfg = wl.C2
    say("C2 seed", seed, "path", path)
    x, z = wl.make(cfg)
    with pk.Picasso(x, z, cfg.q) as h:
        h.set_option(pk.OPT_PAIR_PATH, path)
        nc, col = h.color(seed, cfg.frac, cfg.alpha, cfg.relation)
        st = h.stats()
    assert nc == g["n_colors"]
    assert col[:32].tolist() == g["colors_head"]
    assert hashlib.sha256(np.ascontiguousarray(col, dtype="<i4").tobytes()).hexdigest() == g["colors_sha256"]
    assert st["n_iters"] == len(g["iters"])
    for a, b in zip(st["iters"], g["iters"]):
        for k in ("m", "P", "T", "pair_tests", "edges", "colored", "offset"):
            assert a[k] == b[k], (k, a[k], b[k])
        if path != pk.PATH_AUTO:
            assert a["pair_path"] == path
    check_valid(x, z, col, cfg.relation)
