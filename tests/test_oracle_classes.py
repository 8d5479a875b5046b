"""Pins for the oracle's edge-free mode (Sec. IV-B static order, Alg. 1).

The edge-free greedy decides each vertex from the colour classes built so
far and the relation: colour c of v's list is forbidden iff some vertex
already coloured c is related to v (such a vertex holds c, so it shares c
with v and the pair is a conflict edge exactly when the relation holds).
These tests tie it to the edge-list greedy, which is itself pinned by the
greedy certificate and the textbook reductions in test_oracle_greedy.py,
and tie the count-only edge enumeration to the stored-edge one.
"""
import numpy as np
import pytest

from paper_2401_06713_amd import workloads as wl


def _instance(n, q, probs, seed):
    return wl.pauli_strings(n, q, probs, seed=seed)


@pytest.mark.parametrize("rel", [0, 1, 2])
@pytest.mark.parametrize("n,q,probs,P,T,seed", [
    (300, 6, (0.25, 0.25, 0.25, 0.25), 40, 5, 1),
    (500, 16, (0.7, 0.1, 0.1, 0.1), 30, 30, 2),   # T = P: every relation pair conflicts
    (800, 40, (0.8, 0.2 / 3, 0.2 / 3, 0.2 / 3), 100, 7, 3),
    (27, 3, (0.0, 1 / 3, 1 / 3, 1 / 3), 8, 2, 4),  # all 27 strings without I, tiny palette
])
def test_class_greedy_equals_edge_greedy(orc, rel, n, q, probs, P, T, seed):
    x, z = _instance(n, q, probs, seed)
    ch = orc.decode(x, z, q)
    ids = np.arange(n, dtype=np.int32)
    lists = orc.sample_lists(seed, 1, ids, P, T)
    prio = orc.priorities(seed, 1, ids)
    edges, cnt, _ = orc.conflict_edges_bucketed(ch, ids, lists, P, rel)
    want = orc.greedy_from_edges(prio, lists, P, edges)
    got = orc.greedy_by_classes(ch, ids, lists, P, prio, rel)
    assert np.array_equal(got, want)


def test_class_greedy_subset_and_ties(orc):
    """A vertex subset (local index != original id) and equal priorities
    (ties broken by local index)."""
    x, z = _instance(600, 12, (0.5, 1 / 6, 1 / 6, 1 / 6), 9)
    ch = orc.decode(x, z, 12)
    ids = np.arange(0, 600, 3, dtype=np.int32)
    lists = orc.sample_lists(4, 2, ids, 25, 4)
    prio = orc.priorities(4, 2, ids)
    prio[::2] = prio[0]
    for rel in (0, 1, 2):
        edges, _, _ = orc.conflict_edges_bucketed(ch, ids, lists, 25, rel)
        assert np.array_equal(orc.greedy_by_classes(ch, ids, lists, 25, prio, rel),
                              orc.greedy_from_edges(prio, lists, 25, edges))


@pytest.mark.parametrize("rel", [0, 1, 2])
def test_count_only_edges_equal_stored_edges(orc, rel):
    x, z = _instance(700, 20, (0.6, 0.4 / 3, 0.4 / 3, 0.4 / 3), 5)
    ch = orc.decode(x, z, 20)
    ids = np.arange(700, dtype=np.int32)
    P, T = 60, 6
    lists = orc.sample_lists(1, 1, ids, P, T)
    edges, cnt, tests = orc.conflict_edges_bucketed(ch, ids, lists, P, rel)
    assert orc.count_conflict_edges(ch, ids, lists, P, rel) == (cnt, tests)
    # slices partition the colours, and with them the edges
    cuts = [0, 7, 31, 32, 60]
    parts = [orc.count_conflict_edges(ch, ids, lists, P, rel, a, b) for a, b in zip(cuts[:-1], cuts[1:])]
    assert sum(c for c, _ in parts) == cnt and sum(t for _, t in parts) == tests
    # the plain all-pairs definition
    assert orc.conflict_edges_allpairs(ch, ids, lists, rel).shape[0] == cnt


@pytest.mark.parametrize("rel", [0, 1, 2])
@pytest.mark.parametrize("n,q,probs,frac,alpha,fixed_T", [
    (1500, 16, (0.25, 0.25, 0.25, 0.25), 0.125, 2.0, 0),
    (2500, 48, (0.7, 0.1, 0.1, 0.1), 0.05, 1.0, 0),
    (900, 30, (0.6, 0.4 / 3, 0.4 / 3, 0.4 / 3), 0.03, 30.0, 0),   # the aggressive preset
    (1200, 20, (0.5, 1 / 6, 1 / 6, 1 / 6), 0.2, 2.0, 3),
])
def test_edge_free_run_equals_edge_run(orc, rel, n, q, probs, frac, alpha, fixed_T):
    x, z = _instance(n, q, probs, 11)
    a = orc.color(x, z, q, 7, frac, alpha, rel, fixed_T=fixed_T)
    b = orc.color_classes(x, z, q, 7, frac, alpha, rel, fixed_T=fixed_T)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and a[2] == b[2]
    c = orc.color_classes(x, z, q, 7, frac, alpha, rel, fixed_T=fixed_T, count_edges=False)
    assert c[0] == a[0] and np.array_equal(c[1], a[1])
    assert all(s["edges"] == -1 for s in c[2])
    assert [{k: v for k, v in s.items() if k != "edges"} for s in c[2]] == \
           [{k: v for k, v in s.items() if k != "edges"} for s in a[2]]


def test_edge_free_schedule_equals_schedule_run(orc):
    x, z = _instance(2000, 24, (0.6, 0.4 / 3, 0.4 / 3, 0.4 / 3), 12)
    fr, al = [0.08, 0.1, 0.2], [1.5, 2.5, 3.0]
    a = orc.color_schedule(x, z, 24, 3, fr, al, 0)
    b = orc.color_classes(x, z, 24, 3, fr, al, 0)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_learned_driver_uses_the_fp64_network(orc):
    """Each iteration's (f, alpha) is the FP64 network on that iteration's
    features, and the run equals the schedule run with those values."""
    x, z = _instance(3000, 32, (0.7, 0.1, 0.1, 0.1), 13)
    rng = np.random.default_rng(0)
    params = rng.normal(0, 0.3, orc.mlp_nparams())
    beta = 0.3
    nc, col, st, sched = orc.color_learned(x, z, 32, 5, params, 0, beta)
    assert sched.shape == (len(st), 2)
    n = x.shape[0]
    for k, s in enumerate(st):
        ids = np.nonzero(col >= s["offset"])[0].astype(np.int32)
        assert ids.shape[0] == s["m"]
        feat = np.r_[orc.features(x, z, 32, ids, 5, k + 1, 0), beta]
        f, a = orc.mlp_squash(orc.mlp_forward(params, feat)[0])
        assert sched[k, 0] == f and sched[k, 1] == a
        assert (s["P"], s["T"]) == orc.params(s["m"], f, a)
    rep = orc.color_schedule(x, z, 32, 5, sched[:, 0], sched[:, 1], 0)
    assert rep[0] == nc and np.array_equal(rep[1], col) and rep[2] == st
    assert col.min() >= 0 and col.shape[0] == n
