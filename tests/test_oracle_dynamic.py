"""Pins for the oracle's dynamic-order list colouring (Alg. 2, Sec. IV-B).

Independent checks: a pure-Python replay of the algorithm's rules from the
order and colours the oracle reports (the next vertex always has the
shortest remaining list, takes a colour still in it, and that colour leaves
exactly the neighbours' lists that held it, emptying some); uniformity of
the random choices; the empty graph; complete graphs with the whole
palette; and validity, list respect and progress on full runs of Alg. 1
with this colourer.
"""
import numpy as np
import pytest
from scipy import stats

from paper_2401_06713_amd import workloads as wl
from tests.test_oracle_greedy import iteration_of, relation_matrix


def random_instance(rng, m, P, T, dens):
    lists = np.sort(np.array([rng.choice(P, T, replace=False) for _ in range(m)]), axis=1).astype(np.uint32)
    e = [(a, b) for a in range(m) for b in range(a + 1, m) if rng.random() < dens]
    return lists, np.array(e, dtype=np.int32).reshape(-1, 2)


def replay(lists, edges, col, order):
    """Re-derive Alg. 2's rules step by step from the reported run."""
    m = lists.shape[0]
    cur = [set(int(c) for c in row) for row in lists]
    nbr = [set() for _ in range(m)]
    for a, b in edges:
        nbr[a].add(int(b))
        nbr[b].add(int(a))
    done = np.zeros(m, dtype=bool)
    assert sorted(order.tolist()) == list(range(m))  # every vertex taken exactly once
    k = 0
    while k < m:
        v = int(order[k])
        assert not done[v] and col[v] >= 0, "a step starts with a vertex that gets a colour"
        live = [len(cur[u]) for u in range(m) if not done[u]]
        assert len(cur[v]) == min(live), "the vertex comes from the lowest bucket"
        c = int(col[v])
        assert c in cur[v], "its colour is still in its list"
        done[v] = True
        k += 1
        emptied = set()
        for u in nbr[v]:
            if not done[u] and c in cur[u]:
                cur[u].discard(c)
                if not cur[u]:
                    emptied.add(u)
        got = set(int(u) for u in order[k:k + len(emptied)])
        assert got == emptied, "neighbours whose lists empty are taken right after, uncoloured"
        for u in emptied:
            assert col[u] == -1
            done[u] = True
        k += len(emptied)
    for a, b in edges:  # proper
        assert not (col[a] >= 0 and col[a] == col[b])


@pytest.mark.parametrize("seed", range(8))
def test_replay_random_graphs(orc, seed):
    rng = np.random.default_rng(200 + seed)
    m = int(rng.integers(1, 160))
    P = int(rng.integers(1, 30))
    T = int(rng.integers(1, P + 1))
    lists, edges = random_instance(rng, m, P, T, float(rng.uniform(0, 0.6)))
    col, order = orc.greedy_dynamic(lists, edges, seed, 1)
    replay(lists, edges, col, order)


def test_first_choices_are_uniform(orc):
    # no edges, equal list sizes: the first vertex is uniform over all, and
    # its colour is uniform over its list
    m, P = 8, 3
    lists = np.tile(np.arange(P, dtype=np.uint32), (m, 1))
    edges = np.zeros((0, 2), np.int32)
    first = np.zeros(m, np.int64)
    colour = np.zeros(P, np.int64)
    for seed in range(4000):
        col, order = orc.greedy_dynamic(lists, edges, seed, 1)
        first[order[0]] += 1
        colour[col[order[0]]] += 1
    assert stats.chisquare(first).pvalue > 1e-3
    assert stats.chisquare(colour).pvalue > 1e-3


def test_empty_graph_colours_everyone_from_its_list(orc):
    rng = np.random.default_rng(5)
    lists, _ = random_instance(rng, 300, 40, 6, 0.0)
    col, order = orc.greedy_dynamic(lists, np.zeros((0, 2), np.int32), 9, 2)
    assert all(int(col[v]) in lists[v].tolist() for v in range(300))


@pytest.mark.parametrize("m,P", [(10, 10), (7, 12), (15, 6)])
def test_complete_graph_full_palette(orc, m, P):
    # complete graph, every list the whole palette: each colour taken leaves
    # every other list, so min(m, P) vertices get distinct colours and the
    # rest empty
    lists = np.tile(np.arange(P, dtype=np.uint32), (m, 1))
    edges = np.array([(a, b) for a in range(m) for b in range(a + 1, m)], np.int32).reshape(-1, 2)
    col, order = orc.greedy_dynamic(lists, edges, 3, 1)
    got = col[col >= 0]
    assert got.size == min(m, P) and np.unique(got).size == got.size
    replay(lists, edges, col, order)


@pytest.mark.parametrize("rel", [0, 1, 2])
def test_full_run_with_dynamic_colourer(orc, rel):
    n, q = 500, 10
    x, z = wl.pauli_strings(n, q, (0.5, 0.2, 0.2, 0.1), seed=31 + rel)
    nc, col, st = orc.color(x, z, q, 6, 0.125, 2.0, rel, dynamic=True)
    R = relation_matrix(orc, x, z, q, rel)
    assert np.all(col >= 0)
    assert not np.any((col[:, None] == col[None, :]) & R)
    assert nc == len(np.unique(col))
    assert all(s["colored"] >= 1 for s in st)
    for a, b in zip(st, st[1:]):
        assert b["offset"] == a["offset"] + a["P"] and b["m"] == a["m"] - a["colored"]
    for v in range(n):  # list respect
        k = iteration_of(st, int(col[v]))
        L = orc.sample_list(6, k + 1, v, st[k]["P"], st[k]["T"])
        assert col[v] - st[k]["offset"] in L.tolist()


# ---------------------------------------------------------------- round form
TAG_DYNK, TAG_DYNC = 0x44594E4B, 0x44594E43


def rounds_replay(orc, ids, lists, edges, seed, ell, divisor):
    """The round form's rules, restated in plain Python (tiny graphs)."""
    m, T = lists.shape
    nbr = [set() for _ in range(m)]
    for a, b in edges:
        nbr[a].add(int(b))
        nbr[b].add(int(a))
    alive = [list(int(c) for c in row) for row in lists]  # ascending remaining colours
    col = [-1] * m
    failed = [False] * m
    rnd = 0
    while True:
        for v in range(m):
            if col[v] < 0 and not failed[v] and not alive[v]:
                failed[v] = True
        act = [v for v in range(m) if col[v] < 0 and not failed[v]]
        if not act:
            return np.array(col, dtype=np.int32), rnd
        A = len(act)
        R = max(-(-A // divisor), min(A, 64))
        sizes = sorted(len(alive[v]) for v in act)
        sstar = sizes[R - 1]
        below = sum(1 for s in sizes if s < sstar)
        eq = sum(1 for s in sizes if s == sstar)
        need = R - below
        cut = 1 << 32 if need >= eq else (need << 32) // eq
        reqs = []
        for v in act:
            s = len(alive[v])
            h = orc.hash64(seed, int(ids[v]), rnd, ell, TAG_DYNK) >> 32
            if s < sstar or (s == sstar and h < cut):
                j = (orc.hash64(seed, int(ids[v]), rnd, ell, TAG_DYNC) * s) >> 64
                reqs.append((alive[v][j], (s << 32) | h, v))
        winners = {}
        for c, key, v in sorted(reqs):
            if not any(winners.get(u) == c for u in nbr[v]):
                winners[v] = c
        for v, c in winners.items():
            col[v] = c
        for v, c in winners.items():
            for u in nbr[v]:
                if c in alive[u]:
                    alive[u].remove(c)
        rnd += 1


@pytest.mark.parametrize("seed", range(6))
def test_round_form_follows_its_rules(orc, seed):
    rng = np.random.default_rng(300 + seed)
    m, P, T = int(rng.integers(20, 90)), int(rng.integers(4, 20)), 0
    T = int(rng.integers(1, min(P, 8) + 1))
    lists, edges = random_instance(rng, m, P, T, float(rng.uniform(0.1, 0.6)))
    ids = np.sort(rng.choice(10_000, m, replace=False)).astype(np.int32)
    divisor = int(rng.choice([1, 2, 4, 16]))
    col, rounds = orc.greedy_dynamic_rounds(ids, lists, edges, seed, 2, divisor)
    ref, ref_rounds = rounds_replay(orc, ids, lists, edges, seed, 2, divisor)
    assert np.array_equal(col, ref) and rounds == ref_rounds


def test_round_form_valid_and_respects_lists(orc):
    rng = np.random.default_rng(7)
    for _ in range(5):
        m, P, T = 400, 60, 6
        lists, edges = random_instance(rng, m, P, T, 0.3)
        ids = np.arange(m, dtype=np.int32)
        col, _ = orc.greedy_dynamic_rounds(ids, lists, edges, 11, 1, 16)
        for a, b in edges:
            assert not (col[a] >= 0 and col[a] == col[b])
        for v in range(m):
            assert col[v] == -1 or col[v] in lists[v]


def test_round_form_special_graphs(orc):
    rng = np.random.default_rng(8)
    m, P, T = 150, 40, 5
    lists = np.sort(np.array([rng.choice(P, T, replace=False) for _ in range(m)]), axis=1).astype(np.uint32)
    ids = np.arange(m, dtype=np.int32)
    # no edges: every vertex takes a colour of its list
    col, _ = orc.greedy_dynamic_rounds(ids, lists, np.zeros((0, 2), np.int32), 3, 1, 16)
    assert (col >= 0).all() and all(col[v] in lists[v] for v in range(m))
    # complete graph, whole palette as every list: each colour at most once,
    # min(m, P) vertices coloured
    full = np.tile(np.arange(P, dtype=np.uint32), (m, 1))
    edges = np.array([(a, b) for a in range(m) for b in range(a + 1, m)], np.int32)
    col, _ = orc.greedy_dynamic_rounds(ids, full, edges, 3, 1, 4)
    c = col[col >= 0]
    assert c.size == min(m, P) and np.unique(c).size == c.size


def test_round_form_keeps_most_of_alg2s_gain(orc):
    """C1, colouring seeds 0-2: whole runs with the round form (divisor 16)
    use fewer colours than the static order and at most 3% more than the
    sequential Alg. 2."""
    cfg = wl.C1
    x, z = wl.make(cfg)
    rf, seq, st = [], [], []
    for seed in range(3):
        rf.append(orc.color(x, z, cfg.q, seed, cfg.frac, cfg.alpha, 0, dynamic=True, rounds_divisor=16)[0])
        seq.append(orc.color(x, z, cfg.q, seed, cfg.frac, cfg.alpha, 0, dynamic=True)[0])
        st.append(orc.color(x, z, cfg.q, seed, cfg.frac, cfg.alpha, 0)[0])
    assert np.mean(rf) < np.mean(st)
    assert np.mean(rf) <= 1.03 * np.mean(seq)
