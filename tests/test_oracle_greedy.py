"""Pins for the oracle's list colouring and iteration (Sec. IV-B static
order schemes; Alg. 1).

Independent checks: proper colouring of the relation graph, list respect,
palette disjointness, progress, the greedy certificate on random graphs,
networkx's textbook greedy when T = P, complete and empty relation graphs,
and the chromatic lower bound by subset DP for n <= 12.
"""
import itertools

import networkx as nx
import numpy as np
import pytest

from paper_2401_06713_amd import workloads as wl


def relation_matrix(orc, x, z, q, rel):
    ch = orc.decode(x, z, q)
    n = ch.shape[0]
    R = np.zeros((n, n), dtype=bool)
    for a in range(n):
        for b in range(a + 1, n):
            R[a, b] = R[b, a] = orc.relation_chars(ch[a].tobytes(), ch[b].tobytes(), rel)
    return R


def check_greedy_certificate(prio, lists, edges, col):
    """The colouring is THE greedy result of the (prio, index) order iff, for
    every vertex v: a coloured v holds a list colour no earlier neighbour
    holds, and every smaller list colour is held by an earlier neighbour; an
    uncoloured v sees every list colour held by an earlier neighbour.  By
    induction over the order these conditions determine the colouring."""
    m, T = lists.shape
    order = sorted(range(m), key=lambda i: (int(prio[i]), i))
    rank = np.empty(m, dtype=np.int64)
    rank[order] = np.arange(m)
    nbr = [[] for _ in range(m)]
    for a, b in edges:
        nbr[a].append(b)
        nbr[b].append(a)
    for v in range(m):
        taken = {int(col[u]) for u in nbr[v] if rank[u] < rank[v] and col[u] >= 0}
        L = [int(c) for c in lists[v]]
        if col[v] >= 0:
            assert col[v] in L and col[v] not in taken
            assert all(c in taken for c in L if c < col[v])
        else:
            assert all(c in taken for c in L)
        for u in nbr[v]:  # proper
            assert not (col[u] >= 0 and col[u] == col[v])


@pytest.mark.parametrize("seed", range(6))
def test_greedy_certificate_random_graphs(orc, seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 300))
    P = int(rng.integers(1, 40))
    T = int(rng.integers(1, P + 1))
    lists = np.sort(np.array([rng.choice(P, T, replace=False) for _ in range(m)]), axis=1).astype(np.uint32)
    dens = rng.uniform(0, 0.5)
    e = [(a, b) for a in range(m) for b in range(a + 1, m) if rng.random() < dens]
    edges = np.array(e, dtype=np.int32).reshape(-1, 2)
    prio = rng.integers(0, 2**63, m, dtype=np.int64).astype(np.uint64)
    if seed % 2:
        prio[: m // 2] = prio[0]  # force ties: broken by index
    col = orc.greedy_from_edges(prio, lists, P, edges)
    check_greedy_certificate(prio, lists, edges, col)


def iteration_of(stats, colour):
    for k, s in enumerate(stats):
        if s["offset"] <= colour < s["offset"] + s["P"]:
            return k
    raise AssertionError("colour outside every palette")


@pytest.mark.parametrize("rel", [0, 1, 2])
@pytest.mark.parametrize("n,q,probs,frac,alpha", [
    (400, 8, (0.25, 0.25, 0.25, 0.25), 0.125, 2.0),
    (600, 30, (0.7, 0.1, 0.1, 0.1), 0.05, 3.0),
    (300, 12, (0.5, 0.2, 0.2, 0.1), 0.25, 1.0),
])
def test_full_run_properties(orc, rel, n, q, probs, frac, alpha):
    x, z = wl.pauli_strings(n, q, probs, seed=n + q)
    nc, col, st = orc.color(x, z, q, 7, frac, alpha, rel)
    R = relation_matrix(orc, x, z, q, rel)
    assert np.all(col >= 0)  # every vertex coloured
    # proper: a colour class holds no relation edge
    same = col[:, None] == col[None, :]
    assert not np.any(same & R)
    assert nc == len(np.unique(col))
    # palettes are disjoint and cumulative
    assert st[0]["offset"] == 0
    for a, b in zip(st, st[1:]):
        assert b["offset"] == a["offset"] + a["P"]
        assert b["m"] == a["m"] - a["colored"]
    assert all(s["colored"] >= 1 for s in st)  # progress
    assert nc <= sum(s["P"] for s in st)
    # list respect: each colour lies in the vertex's list of its iteration
    for v in range(n):
        k = iteration_of(st, int(col[v]))
        s = st[k]
        L = orc.sample_list(7, k + 1, v, s["P"], s["T"])
        assert col[v] - s["offset"] in L.tolist()
    # the first vertex of iteration 1's order takes its smallest list colour
    pr = [orc.priority(7, 1, v) for v in range(n)]
    v0 = min(range(n), key=lambda i: (pr[i], i))
    assert col[v0] == orc.sample_list(7, 1, v0, st[0]["P"], st[0]["T"])[0]


@pytest.mark.parametrize("rel", [0, 1, 2])
def test_full_palette_is_textbook_greedy(orc, rel):
    # T = P = m >= Delta + 1: one iteration, and the list colouring is the
    # classical greedy colouring in the random order.
    n, q = 150, 6
    x, z = wl.pauli_strings(n, q, seed=rel + 40)
    nc, col, st = orc.color(x, z, q, 3, 1.0, 1.0, rel, fixed_T=10**6)
    assert len(st) == 1 and st[0]["P"] == n and st[0]["T"] == n
    R = relation_matrix(orc, x, z, q, rel)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(*np.nonzero(np.triu(R))))
    pr = [orc.priority(3, 1, v) for v in range(n)]
    order = sorted(range(n), key=lambda i: (pr[i], i))
    ref = nx.coloring.greedy_color(G, strategy=lambda g, colors: iter(order))
    assert [ref[v] for v in range(n)] == col.tolist()
    assert nc == max(ref.values()) + 1


@pytest.mark.parametrize("q", [4, 9, 33])
def test_complete_relation_needs_n_colours(orc, q):
    x, z = wl.majorana_strings(q)
    nc, col, st = orc.color(x, z, q, 1, 0.125, 2.0, 0)
    assert nc == 2 * q and len(np.unique(col)) == 2 * q


@pytest.mark.parametrize("q", [4, 9, 33])
def test_commute_relation_on_majorana_strings_is_empty(orc, q):
    # the 2q Majorana strings pairwise anticommute: under COMMUTE no pair is
    # an edge, so one iteration colours every string with its first list colour
    x, z = wl.majorana_strings(q)
    nc, col, st = orc.color(x, z, q, 4, 0.125, 2.0, 2)
    assert len(st) == 1 and st[0]["edges"] == 0
    P, T = st[0]["P"], st[0]["T"]
    assert col.tolist() == [int(orc.sample_list(4, 1, v, P, T)[0]) for v in range(2 * q)]


def test_commute_relation_on_iz_strings_is_complete(orc):
    # strings over {I, Z} pairwise commute: under COMMUTE every pair is an
    # edge and every string needs a colour of its own
    n, q = 120, 12
    x, z = wl.iz_strings(n, q, seed=9)
    nc, col, st = orc.color(x, z, q, 2, 0.125, 2.0, 2)
    assert nc == n and len(np.unique(col)) == n


def test_commute_classes_pairwise_anticommute(orc):
    # every colour class under COMMUTE is a set of mutually anticommuting
    # strings, checked on the Pauli matrices themselves
    from tests.test_oracle_relation import kron_string
    q = 3
    x, z = wl.pauli_strings(63, q, seed=4)  # all 63 non-identity strings
    ch = orc.decode(x, z, q)
    mats = [kron_string(bytes(r).decode()) for r in ch]
    for cseed in range(3):
        nc, col, _ = orc.color(x, z, q, cseed, 0.125, 2.0, 2)
        for c in np.unique(col):
            members = np.flatnonzero(col == c)
            for a, b in itertools.combinations(members, 2):
                assert np.allclose(mats[a] @ mats[b] + mats[b] @ mats[a], 0)


def test_aggressive_preset_full_lists(orc):
    # the paper's aggressive setting (palette 3% of |V|, list size 30 ln|V|)
    # gives T = P at this size: every pair shares the palette, so the first
    # iteration is the textbook greedy colouring over P colours
    n, q = 400, 8
    x, z = wl.pauli_strings(n, q, seed=12)
    nc, col, st = orc.color(x, z, q, 1, 0.03, 30.0, 2)
    assert st[0]["P"] == 12 and st[0]["T"] == 12
    R = relation_matrix(orc, x, z, q, 2)
    assert not np.any((col[:, None] == col[None, :]) & R)
    assert np.all(col >= 0)


def test_empty_relation_single_iteration(orc):
    n, q = 500, 16
    x, z = wl.iz_strings(n, q, seed=2)
    for rel in (0, 1):
        nc, col, st = orc.color(x, z, q, 5, 0.125, 2.0, rel)
        assert len(st) == 1 and st[0]["edges"] == 0
        P, T = st[0]["P"], st[0]["T"]
        mins = [int(orc.sample_list(5, 1, v, P, T)[0]) for v in range(n)]
        assert col.tolist() == mins
        assert nc == len(set(mins))


def chromatic_number(R):
    n = R.shape[0]
    adj = [sum(1 << j for j in range(n) if R[i, j]) for i in range(n)]
    indep = [True] * (1 << n)
    for s in range(1, 1 << n):
        low = (s & -s).bit_length() - 1
        rest = s & ~(1 << low)
        indep[s] = indep[rest] and not (adj[low] & rest)
    INF = n + 1
    dp = [INF] * (1 << n)
    dp[0] = 0
    for s in range(1, 1 << n):
        sub = s
        best = INF
        while sub:
            if indep[sub] and dp[s & ~sub] + 1 < best:
                best = dp[s & ~sub] + 1
            sub = (sub - 1) & s
        dp[s] = best
    return dp[(1 << n) - 1]


@pytest.mark.parametrize("seed", range(4))
def test_chromatic_lower_bound_small(orc, seed):
    n, q = 11, 4
    x, z = wl.pauli_strings(n, q, seed=seed)
    for rel in (0, 1, 2):
        R = relation_matrix(orc, x, z, q, rel)
        chi = chromatic_number(R)
        for cseed in range(3):
            nc, col, _ = orc.color(x, z, q, cseed, 0.125, 2.0, rel)
            assert nc >= chi


def test_trivial_sizes(orc):
    x, z = wl.pauli_strings(1, 5, seed=0)
    nc, col, st = orc.color(x, z, 5, 0, 0.125, 2.0, 0)
    assert nc == 1 and col.tolist() == [0] and len(st) == 1
    nc, col, st = orc.color(np.zeros((0, 1), np.uint64), np.zeros((0, 1), np.uint64), 5, 0, 0.125, 2.0, 0)
    assert nc == 0 and st == []
    # two anticommuting strings: X and Z
    x = np.array([[1], [0]], np.uint64)
    z = np.array([[0], [1]], np.uint64)
    nc, col, st = orc.color(x, z, 1, 0, 0.125, 2.0, 0)
    assert nc == 2 and col[0] != col[1]


def test_duplicates_accepted(orc):
    # identical strings commute and are QWC: no edge between them
    x, z = wl.pauli_strings(50, 6, seed=1)
    x2 = np.concatenate([x, x[:10]])
    z2 = np.concatenate([z, z[:10]])
    for rel in (0, 1, 2):
        nc, col, st = orc.color(x2, z2, 6, 2, 0.125, 2.0, rel)
        R = relation_matrix(orc, x2, z2, 6, rel)
        assert not np.any((col[:, None] == col[None, :]) & R)
