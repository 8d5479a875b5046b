"""HIP path vs the CPU oracle, element by element, through the C ABI.

All integer work: the bar is bit-exact.  Conflict-graph rows come back
unordered (the order of edges inside a CSR row carries no meaning), so
edge sets are compared in canonical sorted form.
"""
import math
import sys

import numpy as np
import pytest

import paper_2401_06713_amd as pk
from paper_2401_06713_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def strings(n, q, probs=(0.25, 0.25, 0.25, 0.25), seed=0):
    return wl.pauli_strings(n, q, probs, seed=seed)


# ---------------------------------------------------------------- lists
@pytest.mark.parametrize("n,q,P,T,ell,sub", [
    (2000, 16, 250, 16, 1, False),      # C1 sizes
    (5000, 48, 25000, 25, 1, False),
    (3000, 20, 300, 64, 2, True),
    (1500, 20, 5000, 65, 3, True),      # 128-thread sampler blocks
    (777, 20, 4000, 256, 5, True),      # 64-thread blocks
    (600, 20, 3000, 300, 2, True),      # 32-thread blocks
    (300, 20, 1500, 1024, 3, False),    # largest T, 16-thread blocks
    (300, 20, 7, 7, 1, False),          # T = P
    (301, 20, 1, 1, 2, False),          # P = 1
])
def test_lists_bit_exact(orc, n, q, P, T, ell, sub):
    say("lists", n, q, P, T, ell, sub)
    x, z = strings(n, q, seed=n)
    ids = np.arange(n, dtype=np.int32)
    if sub:
        ids = np.sort(np.random.default_rng(1).choice(n, n // 2 + 1, replace=False)).astype(np.int32)
    with pk.Picasso(x, z, q) as h:
        lists, prio = h.sample_lists(12345, ell, ids, P, T)
    ref = orc.sample_lists(12345, ell, ids, P, T)
    assert np.array_equal(lists, ref)
    ref_prio = orc.priorities(12345, ell, ids)
    assert np.array_equal(prio, ref_prio)


# ---------------------------------------------------------------- conflict graph
def gpu_edges(h, seed, ell, ids, P, T, rel):
    rowptr, adj = h.conflict_graph(seed, ell, ids, P, T, rel)
    e = pk.edges_from_csr(rowptr, adj)
    # symmetric and duplicate-free rows
    deg = np.diff(rowptr)
    assert deg.sum() == 2 * len(e)
    assert len(np.unique(e, axis=0)) == len(e)
    return e


_ORACLE_EDGES = {}


@pytest.mark.parametrize("path", [pk.PATH_VALU, pk.PATH_MFMA])
@pytest.mark.parametrize("rel", [0, 1, 2])
@pytest.mark.parametrize("n,q,probs,P,T", [
    (2000, 16, (0.25, 0.25, 0.25, 0.25), 250, 16),    # C1 iteration 1
    (1500, 48, (0.7, 0.1, 0.1, 0.1), 120, 20),
    (1200, 100, (0.8, 0.2 / 3, 0.2 / 3, 0.2 / 3), 60, 14),  # W = 2
    (900, 150, (0.8, 0.2 / 3, 0.2 / 3, 0.2 / 3), 40, 9),    # W = 3
    (800, 256, (0.85, 0.05, 0.05, 0.05), 30, 8),             # W = 4
    (1100, 30, (0.6, 0.1, 0.2, 0.1), 2, 1),                 # buckets > 512 members (column chunks)
    (700, 64, (0.5, 0.2, 0.2, 0.1), 9000, 3),               # mostly empty buckets
    (3000, 40, (0.7, 0.1, 0.1, 0.1), 6, 3),                  # buckets > 1024 members: exact dedup path
    (1500, 24, (0.6, 0.1, 0.2, 0.1), 100, 64),              # long prefixes: several hash passes
    (1200, 24, (0.6, 0.1, 0.2, 0.1), 300, 200),             # T near the limit, multi-word slot masks
])
def test_conflict_graph_bit_exact(orc, path, rel, n, q, probs, P, T):
    say("graph", path, rel, n, q, P, T)
    x, z = strings(n, q, probs, seed=q)
    ids = np.sort(np.random.default_rng(q).choice(n, n - n // 5, replace=False)).astype(np.int32)
    with pk.Picasso(x, z, q) as h:
        h.set_option(pk.OPT_PAIR_PATH, path)
        got = gpu_edges(h, 99, 2, ids, P, T, rel)
    key = (rel, n, q, P, T)
    if key not in _ORACLE_EDGES:
        ch = orc.decode(x, z, q)
        lists = orc.sample_lists(99, 2, ids, P, T)
        _ORACLE_EDGES[key] = orc.conflict_edges_bucketed(ch, ids, lists, P, rel)[:2]
    ref, cnt = _ORACLE_EDGES[key]
    assert cnt == len(got)
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- list colouring
@pytest.mark.parametrize("seed", range(5))
def test_jp_equals_sequential_greedy(orc, seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(50, 4000))
    P = int(rng.integers(1, 200))
    T = int(rng.integers(1, min(P, 130) + 1))
    lists = np.sort(np.array([rng.choice(P, T, replace=False) for _ in range(m)]), axis=1).astype(np.uint32)
    k = int(rng.integers(0, min(m * 30, 200_000)))
    a = rng.integers(0, m, k)
    b = rng.integers(0, m, k)
    e = np.unique(np.stack([np.minimum(a, b), np.maximum(a, b)], 1)[a != b], axis=0).astype(np.int32)
    prio = rng.integers(0, 2**63, m, dtype=np.int64).astype(np.uint64)
    if seed == 3:
        prio[:] = 5  # all tied: order by index
    say("jp", m, P, T, len(e))
    ref = orc.greedy_from_edges(prio, lists, P, e)
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    order = np.argsort(src, kind="stable")
    rowptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(src, minlength=m), out=rowptr[1:])
    got = pk.list_color_csr(prio, lists, P, rowptr, dst[order])
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- whole method
def run_both(orc, x, z, q, seed, frac, alpha, rel, fixed_T=0, path=pk.PATH_AUTO, bucket_build=0):
    with pk.Picasso(x, z, q) as h:
        h.set_option(pk.OPT_PAIR_PATH, path)
        h.set_option(pk.OPT_BUCKET_BUILD, bucket_build)
        if fixed_T:
            h.set_option(pk.OPT_FIXED_T, fixed_T)
        nc, col = h.color(seed, frac, alpha, rel)
        st = h.stats()
    rnc, rcol, rst = orc.color(x, z, q, seed, frac, alpha, rel, fixed_T=fixed_T)
    assert nc == rnc
    assert np.array_equal(col, rcol)
    assert st["n_iters"] == len(rst)
    for a, b in zip(st["iters"], rst):
        for k in ("m", "P", "T", "pair_tests", "edges", "colored", "offset"):
            assert a[k] == b[k], (k, a[k], b[k])
    return nc, col, st


def test_c1_bit_exact(orc):
    say("C1")
    cfg = wl.C1
    x, z = wl.make(cfg)
    for seed in range(3):
        run_both(orc, x, z, cfg.q, seed, cfg.frac, cfg.alpha, cfg.relation)


@pytest.mark.parametrize("rel", [0, 1, 2])
@pytest.mark.parametrize("n,q,probs,frac,alpha", [
    (5000, 48, (0.7, 0.1, 0.1, 0.1), 0.125, 2.0),
    (3000, 100, (0.8, 0.2 / 3, 0.2 / 3, 0.2 / 3), 0.05, 3.0),
    (2500, 200, (0.75, 0.25 / 3, 0.25 / 3, 0.25 / 3), 0.25, 1.0),
    (4000, 24, (0.5, 0.2, 0.2, 0.1), 0.02, 4.0),
    (999, 64, (0.85, 0.05, 0.05, 0.05), 1.0, 0.5),
])
def test_color_bit_exact(orc, rel, n, q, probs, frac, alpha):
    say("color", rel, n, q, frac, alpha)
    x, z = strings(n, q, probs, seed=n + rel)
    for path in (pk.PATH_VALU, pk.PATH_MFMA):
        run_both(orc, x, z, q, 5, frac, alpha, rel, path=path)


@pytest.mark.parametrize("path", [pk.PATH_VALU, pk.PATH_MFMA])
def test_commute_relation_special_cases(orc, path):
    """COMMUTE (the paper's own orientation): Majorana strings pairwise
    anticommute, so their graph is empty and one iteration gives every string
    its first list colour; {I, Z} strings pairwise commute, so every string
    needs its own colour; the aggressive preset (palette 3% of |V|, list
    size 30 ln|V|) matches the oracle bit for bit."""
    say("commute special cases", path)
    for q in (9, 33, 100):
        x, z = wl.majorana_strings(q)
        nc, col, st = run_both(orc, x, z, q, 4, 0.125, 2.0, 2, path=path)
        assert st["n_iters"] == 1 and st["iters"][0]["edges"] == 0
    x, z = wl.iz_strings(300, 16, seed=9)
    nc, _, _ = run_both(orc, x, z, 16, 2, 0.125, 2.0, 2, path=path)
    assert nc == 300
    x, z = strings(1200, 24, (0.6, 0.1, 0.2, 0.1), seed=77)  # buckets of every string: exact dedup path
    run_both(orc, x, z, 24, 1, 0.03, 30.0, 2, path=path)


def test_edge_cases(orc):
    say("edge cases")
    # one string
    x, z = strings(1, 7)
    run_both(orc, x, z, 7, 0, 0.125, 2.0, 0)
    # two anticommuting strings
    run_both(orc, np.array([[1], [0]], np.uint64), np.array([[0], [1]], np.uint64), 1, 0, 0.125, 2.0, 0)
    # complete graph: Jordan-Wigner Majoranas
    x, z = wl.majorana_strings(40)
    nc, _, _ = run_both(orc, x, z, 40, 1, 0.125, 2.0, 0)
    assert nc == 80
    # empty graph
    x, z = wl.iz_strings(600, 16, seed=3)
    for rel in (0, 1):
        run_both(orc, x, z, 16, 2, 0.125, 2.0, rel)
    # duplicates
    x, z = strings(300, 10, seed=4)
    x2, z2 = np.concatenate([x, x[:50]]), np.concatenate([z, z[:50]])
    for rel in (0, 1, 2):  # under COMMUTE, duplicates conflict
        run_both(orc, x2, z2, 10, 3, 0.125, 2.0, rel)
    # fixed T and the full palette
    x, z = strings(400, 12, seed=6)
    run_both(orc, x, z, 12, 4, 1.0, 1.0, 0, fixed_T=256)
    run_both(orc, x, z, 12, 4, 0.3, 1.0, 1, fixed_T=3)


@pytest.mark.parametrize("build", [1, 2])
@pytest.mark.parametrize("n,q,probs,rel,frac,alpha,fixed_T", [
    (5000, 48, (0.7, 0.1, 0.1, 0.1), 0, 0.125, 2.0, 0),
    (3000, 100, (0.8, 0.2 / 3, 0.2 / 3, 0.2 / 3), 1, 0.05, 3.0, 0),
    (2500, 24, (0.5, 0.2, 0.2, 0.1), 2, 0.01, 4.0, 0),   # buckets above 2048 members
    (1500, 30, (0.7, 0.1, 0.1, 0.1), 0, 0.8, 1.0, 300),  # 16-bit slots
])
def test_bucket_builds_bit_exact(orc, build, n, q, probs, rel, frac, alpha, fixed_T):
    """Both colour-bucket builds (atomics with per-bucket sorts; the radix
    sort by priority then colour) give the oracle's whole run."""
    say("bucket build", build, n, q, rel, frac, alpha, fixed_T)
    x, z = strings(n, q, probs, seed=n + 3 * rel)
    run_both(orc, x, z, q, 2, frac, alpha, rel, fixed_T=fixed_T, bucket_build=build)


def test_long_lists(orc):
    """Lists longer than 256 colours (slot indices past one byte): whole runs
    bit-exact, the slot-wise colouring across several mask words."""
    say("long lists")
    x, z = strings(1500, 30, (0.7, 0.1, 0.1, 0.1), seed=15)
    for rel in (0, 2):
        run_both(orc, x, z, 30, 7, 0.8, 1.0, rel, fixed_T=300)
    x, z = strings(600, 20, seed=16)
    run_both(orc, x, z, 20, 8, 1.0, 1.0, 1, fixed_T=520)


def test_edges_off_same_colours(orc):
    """PICASSO_OPT_EDGES = 0 builds only the relation matrices: the colours
    and iteration sizes are those of the full run, the edge counts -1."""
    x, z = strings(6000, 48, (0.7, 0.1, 0.1, 0.1), seed=17)
    with pk.Picasso(x, z, 48) as h:
        nc, col = h.color(2, 0.125, 2.0, 0)
        st = h.stats()
        h.set_option(pk.OPT_EDGES, 0)
        nc0, col0 = h.color(2, 0.125, 2.0, 0)
        st0 = h.stats()
    assert nc0 == nc and np.array_equal(col0, col)
    for a, b in zip(st0["iters"], st["iters"]):
        for k in ("m", "P", "T", "pair_tests", "colored", "offset"):
            assert a[k] == b[k]
        assert a["edges"] == -1 or a["pair_path"] == 0


def test_aggressive_preset_commute(orc):
    """The paper's aggressive setting (palette 3% of |V|, list size 30 ln|V|)
    under COMMUTE at n = 20,000 (lists of 298 colours over 600, buckets of
    about 10,000 members): colours and iteration sizes bit-exact against the
    oracle's edge-free colouring (edge statistics off on both sides)."""
    n, q = 20000, 48
    x, z = strings(n, q, (0.7, 0.1, 0.1, 0.1), seed=18)
    with pk.Picasso(x, z, q) as h:
        h.set_option(pk.OPT_EDGES, 0)
        nc, col = h.color(3, 0.03, 30.0, 2)
        st = h.stats()
    say("aggressive preset", nc, "colours", st["n_iters"], "iterations", st["iters"][0]["T"], "first T")
    assert st["iters"][0]["T"] == 298
    rnc, rcol, rst = orc.color_classes(x, z, q, 3, 0.03, 30.0, 2, count_edges=False)
    assert nc == rnc and np.array_equal(col, rcol)
    assert st["n_iters"] == len(rst)
    for a, b in zip(st["iters"], rst):
        for k in ("m", "P", "T", "colored", "offset"):
            assert a[k] == b[k], (k, a[k], b[k])


def test_empty_input():
    with pk.Picasso(np.zeros((0, 1), np.uint64), np.zeros((0, 1), np.uint64), 5) as h:
        nc, col = h.color(0, 0.125, 2.0, 0)
        assert nc == 0 and col.size == 0


def test_invalid_arguments():
    x, z = strings(10, 5)
    bad = x.copy()
    bad[0, 0] |= np.uint64(1) << np.uint64(40)  # padding bit
    with pytest.raises(pk.PicassoError):
        pk.Picasso(bad, z, 5)
    with pytest.raises(pk.PicassoError):
        pk.Picasso(x, z, 0)
    with pk.Picasso(x, z, 5) as h:
        for args in ((0, 0.0, 2.0, 0), (0, 1.5, 2.0, 0), (0, 0.1, 0.0, 0), (0, 0.1, 2.0, 7)):
            with pytest.raises(pk.PicassoError) as ei:
                h.color(*args)
            assert ei.value.code == pk.EINVAL
        with pytest.raises(pk.PicassoError):
            h.set_option(99, 1)


def test_memory_budget(orc):
    x, z = strings(3000, 16)
    with pk.Picasso(x, z, 16) as h:
        nc0, col0 = h.color(0, 0.125, 2.0, 0)
        e0 = h.stats()["edges"]
        e1 = h.stats()["iters"][0]["edges"]
        ids = np.arange(h.n, dtype=np.int32)
        P, T = orc.params(h.n, 0.125, 2.0)
        rp0, adj0 = h.conflict_graph(0, 1, ids, P, T, 0)
        assert 2 * e1 == adj0.shape[0] and adj0.nbytes > 16 * 65536
        h.set_option(pk.OPT_MEM_BUDGET, 65536)
        # the CSR is written in chunks of whole rows of at most 64 KiB (more
        # than 16 of them): the same row pointers and adjacency
        rp, adj = h.conflict_graph(0, 1, ids, P, T, 0)
        assert np.array_equal(rp, rp0) and np.array_equal(adj, adj0)
        assert h.conflict_rowptr(0, 1, ids, P, T, 0)[0] == e1
        # the colouring does not need the CSR: same colours, edges still counted
        nc, col = h.color(0, 0.125, 2.0, 0)
        assert nc == nc0 and np.array_equal(col, col0) and h.stats()["edges"] == e0
        # a budget below the longest row cannot be met
        h.set_option(pk.OPT_MEM_BUDGET, 4 * (int(np.diff(rp0).max()) - 1))
        with pytest.raises(pk.PicassoError) as ei:
            h.conflict_graph(0, 1, ids, P, T, 0)
        assert ei.value.code == pk.ENOMEM
        h.set_option(pk.OPT_MEM_BUDGET, 0)


def test_device_io_matches_host_io(orc):
    import torch

    x, z = strings(3000, 40, (0.7, 0.1, 0.1, 0.1), seed=9)
    with pk.Picasso(x, z, 40) as h:
        nc, col = h.color(7, 0.125, 2.0, 0)
    xd = torch.from_numpy(x.view(np.int64)).cuda()
    zd = torch.from_numpy(z.view(np.int64)).cuda()
    out = torch.empty(3000, dtype=torch.int32, device="cuda")
    with pk.Picasso(xd, zd, 40) as h:
        nc2 = h.color_device(out, 7, 0.125, 2.0, 0)
    assert nc2 == nc
    assert np.array_equal(out.cpu().numpy(), col)


def test_repeat_calls_deterministic():
    x, z = strings(4000, 32, (0.7, 0.1, 0.1, 0.1), seed=10)
    with pk.Picasso(x, z, 32) as h:
        a = h.color(3, 0.125, 2.0, 1)
        b = h.color(3, 0.125, 2.0, 1)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
