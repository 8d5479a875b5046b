"""Pins for the oracle's conflict graph (Alg. 1 construct_conflict_graph,
Sec. IV-A: a relation edge is conflicting when the endpoints' lists share a
colour).

Independent checks: a pure-Python brute force built on Kronecker products
for tiny inputs, the T = P special case (every relation edge conflicts), and
the closed-form expectation of |E_c| for i.i.d. strings.
"""
import itertools
import math

import numpy as np
import pytest

from paper_2401_06713_amd import workloads as wl
from tests.test_oracle_relation import SIGMA, kron_string


def brute_edges(strings, lists, rel):
    mats = [kron_string(s) for s in strings]
    out = []
    for a, b in itertools.combinations(range(len(strings)), 2):
        if not set(lists[a].tolist()) & set(lists[b].tolist()):
            continue
        if rel == 0:
            r = np.allclose(mats[a] @ mats[b] + mats[b] @ mats[a], 0)
        elif rel == 2:
            r = np.allclose(mats[a] @ mats[b] - mats[b] @ mats[a], 0)
        else:
            r = not all(np.allclose(SIGMA[s] @ SIGMA[t], SIGMA[t] @ SIGMA[s]) for s, t in zip(strings[a], strings[b]))
        if r:
            out.append((a, b))
    return np.array(out, dtype=np.int32).reshape(-1, 2)


@pytest.mark.parametrize("rel", [0, 1, 2])
@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_vs_brute_force(orc, rel, seed):
    q, n = 3, 36
    x, z = wl.pauli_strings(n, q, seed=seed)
    ch = orc.decode(x, z, q)
    strings = [bytes(r).decode() for r in ch]
    ids = np.arange(n, dtype=np.int32)
    P, T = 9, 3
    lists = orc.sample_lists(seed, 1, ids, P, T)
    ref = brute_edges(strings, lists, rel)
    got = orc.conflict_edges_allpairs(ch, ids, lists, rel)
    assert np.array_equal(got, ref)
    gb, cnt, tests = orc.conflict_edges_bucketed(ch, ids, lists, P, rel)
    assert cnt == len(ref) and np.array_equal(gb, ref)
    counts = np.bincount(lists.ravel(), minlength=P)
    assert tests == int((counts * (counts - 1) // 2).sum())


@pytest.mark.parametrize("rel", [0, 1, 2])
@pytest.mark.parametrize("n,q,P,T,probs", [
    (1200, 16, 150, 14, (0.25, 0.25, 0.25, 0.25)),
    (900, 70, 40, 12, (0.7, 0.1, 0.1, 0.1)),
    (700, 130, 7, 5, (0.8, 0.2 / 3, 0.2 / 3, 0.2 / 3)),
    (500, 24, 600, 3, (0.5, 0.2, 0.2, 0.1)),
])
def test_bucketed_equals_allpairs(orc, rel, n, q, P, T, probs):
    x, z = wl.pauli_strings(n, q, probs, seed=n)
    ch = orc.decode(x, z, q)
    # a subset of vertices, as in a later iteration
    ids = np.sort(np.random.default_rng(n).choice(n, size=n * 3 // 4, replace=False)).astype(np.int32)
    lists = orc.sample_lists(3, 2, ids, P, T)
    a = orc.conflict_edges_allpairs(ch, ids, lists, rel)
    b, cnt, _ = orc.conflict_edges_bucketed(ch, ids, lists, P, rel)
    assert cnt == len(a)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("rel", [0, 1, 2])
def test_full_lists_give_relation_graph(orc, rel):
    # T = P: every pair shares the whole palette, so E_c = relation edges
    q, n, P = 10, 300, 4
    x, z = wl.pauli_strings(n, q, seed=21)
    ch = orc.decode(x, z, q)
    ids = np.arange(n, dtype=np.int32)
    lists = orc.sample_lists(0, 1, ids, P, P)
    e, cnt, tests = orc.conflict_edges_bucketed(ch, ids, lists, P, rel)
    rel_edges = [(a, b) for a, b in itertools.combinations(range(n), 2)
                 if orc.relation_chars(ch[a].tobytes(), ch[b].tobytes(), rel)]
    assert cnt == len(rel_edges)
    assert [tuple(r) for r in e.tolist()] == rel_edges
    assert tests == P * math.comb(n, 2)


def rho(probs, q, rel):
    pI, pX, pY, pZ = probs
    nonI = {"X": pX, "Y": pY, "Z": pZ}
    p = sum(nonI[a] * nonI[b] for a in nonI for b in nonI if a != b)
    if rel == 0:
        return (1 - (1 - 2 * p) ** q) / 2
    if rel == 2:  # commute: an even number of anticommuting positions
        return (1 + (1 - 2 * p) ** q) / 2
    return 1 - (1 - p) ** q


@pytest.mark.parametrize("rel,probs,q", [
    (0, (0.25, 0.25, 0.25, 0.25), 16),
    (0, (0.7, 0.1, 0.1, 0.1), 48),
    (1, (0.85, 0.05, 0.05, 0.05), 48),  # q large enough that duplicate rejection is negligible
    (2, (0.7, 0.1, 0.1, 0.1), 48),
])
def test_expected_conflict_edges(orc, rel, probs, q):
    # E|E_c| = C(n,2) rho (1 - C(P-T,T)/C(P,T)) for i.i.d. positions
    n = 2000
    x, z = wl.pauli_strings(n, q, probs, seed=31)
    ch = orc.decode(x, z, q)
    ids = np.arange(n, dtype=np.int32)
    P, T = orc.params(n, 0.125, 2.0)
    got = []
    for seed in range(3):
        lists = orc.sample_lists(seed, 1, ids, P, T)
        _, cnt, _ = orc.conflict_edges_bucketed(ch, ids, lists, P, rel, want_edges=False)
        got.append(cnt)
    share = 1 - math.comb(P - T, T) / math.comb(P, T)
    expect = math.comb(n, 2) * rho(probs, q, rel) * share
    assert abs(np.mean(got) / expect - 1) < 0.03, (np.mean(got), expect)


def test_colour_slice_partitions_edges(orc):
    q, n = 16, 800
    x, z = wl.pauli_strings(n, q, seed=2)
    ch = orc.decode(x, z, q)
    ids = np.arange(n, dtype=np.int32)
    P, T = 100, 10
    lists = orc.sample_lists(4, 1, ids, P, T)
    full, cnt, tests = orc.conflict_edges_bucketed(ch, ids, lists, P, 0)
    parts = [orc.conflict_edges_bucketed(ch, ids, lists, P, 0, lo, lo + 25) for lo in range(0, P, 25)]
    assert sum(p[1] for p in parts) == cnt
    assert sum(p[2] for p in parts) == tests
    merged = np.concatenate([p[0] for p in parts])
    merged = merged[np.lexsort((merged[:, 1], merged[:, 0]))]
    assert np.array_equal(merged, full)
