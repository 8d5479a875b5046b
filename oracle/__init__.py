"""Plain CPU oracle for the Picasso palette-colouring hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything here.

The arithmetic lives in ``oracle.c`` (single-threaded C, built with gcc into
``liboracle.so``); this module only marshals numpy arrays through ctypes.
See the header of ``oracle.c`` for what pins each function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

REL_ANTICOMMUTE = 0
REL_QWC = 1
REL_COMMUTE = 2


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class IterStat(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("P", ctypes.c_int64),
        ("T", ctypes.c_int64),
        ("pair_tests", ctypes.c_int64),
        ("edges", ctypes.c_int64),
        ("colored", ctypes.c_int64),
        ("offset", ctypes.c_int64),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        i32, i64, u32, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.orc_decode.argtypes = [i64, i32, p, p, p]
        L.orc_decode.restype = None
        L.orc_qubit_anticommutes.argtypes = [ctypes.c_char, ctypes.c_char]
        L.orc_qubit_anticommutes.restype = ctypes.c_int
        L.orc_relation_chars.argtypes = [i32, p, p, i32]
        L.orc_relation_chars.restype = ctypes.c_int
        L.orc_philox4x32_10.argtypes = [p, p, p]
        L.orc_philox4x32_10.restype = None
        L.orc_hash64.argtypes = [u64, u32, u32, u32, u32]
        L.orc_hash64.restype = u64
        L.orc_params.argtypes = [i64, dbl, dbl, i32, p, p]
        L.orc_params.restype = None
        L.orc_sample_list.argtypes = [u64, u32, u32, i64, i32, p]
        L.orc_sample_list.restype = None
        L.orc_priority.argtypes = [u64, u32, u32]
        L.orc_priority.restype = u64
        L.orc_sample_lists.argtypes = [u64, u32, i64, p, i64, i32, p]
        L.orc_sample_lists.restype = None
        L.orc_conflict_edges_allpairs.argtypes = [i32, i64, p, p, p, i32, i32, p, i64]
        L.orc_conflict_edges_allpairs.restype = i64
        L.orc_conflict_edges_bucketed.argtypes = [i32, i64, p, p, p, i32, i64, i32, i64, i64, p, i64, p]
        L.orc_conflict_edges_bucketed.restype = i64
        L.orc_greedy_list_color.argtypes = [i64, p, p, i32, i64, p, p, p]
        L.orc_greedy_list_color.restype = i32
        L.orc_greedy_from_edges.argtypes = [i64, p, p, i32, i64, p, i64, p]
        L.orc_greedy_from_edges.restype = i32
        L.orc_color.argtypes = [i64, i32, p, p, u64, dbl, dbl, i32, i32, p, p, i32, p]
        L.orc_color.restype = i64
        L.orc_color_dynamic.argtypes = [i64, i32, p, p, u64, dbl, dbl, i32, i32, p, p, i32, p]
        L.orc_color_dynamic.restype = i64
        L.orc_greedy_dynamic.argtypes = [i64, p, i32, p, i64, u64, u32, p, p]
        L.orc_greedy_dynamic.restype = i64
        L.orc_greedy_dynamic_rounds.argtypes = [i64, p, p, i32, p, i64, u64, u32, i32, p, p]
        L.orc_greedy_dynamic_rounds.restype = i64
        L.orc_color_dynamic_rounds.argtypes = [i64, i32, p, p, u64, dbl, dbl, i32, i32, i32, p, p, i32, p]
        L.orc_color_dynamic_rounds.restype = i64
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _words(q: int) -> int:
    return (q + 63) // 64


def decode(x: np.ndarray, z: np.ndarray, q: int) -> np.ndarray:
    """Decode bit-plane strings into an (n, q) array of b'I','X','Y','Z'."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    n = x.shape[0]
    out = np.zeros((n, q), dtype=np.uint8)
    lib().orc_decode(n, q, _ptr(x), _ptr(z), _ptr(out))
    return out


def qubit_anticommutes(a: str, b: str) -> bool:
    return bool(lib().orc_qubit_anticommutes(a.encode(), b.encode()))


def relation_chars(a: bytes, b: bytes, rel: int) -> bool:
    assert len(a) == len(b)
    A = np.frombuffer(a, dtype=np.uint8).copy()
    B = np.frombuffer(b, dtype=np.uint8).copy()
    return bool(lib().orc_relation_chars(len(a), _ptr(A), _ptr(B), rel))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def hash64(seed: int, v: int, s: int, ell: int, tag: int) -> int:
    return int(lib().orc_hash64(seed, v, s, ell, tag))


def params(m: int, frac: float, alpha: float, fixed_T: int = 0):
    P = ctypes.c_int64()
    T = ctypes.c_int32()
    lib().orc_params(m, frac, alpha, fixed_T, ctypes.byref(P), ctypes.byref(T))
    return P.value, T.value


def sample_list(seed: int, ell: int, v: int, P: int, T: int) -> np.ndarray:
    out = np.zeros(T, dtype=np.uint32)
    lib().orc_sample_list(seed, ell, v, P, T, _ptr(out))
    return out


def sample_lists(seed: int, ell: int, ids: np.ndarray, P: int, T: int) -> np.ndarray:
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    out = np.zeros((ids.shape[0], T), dtype=np.uint32)
    lib().orc_sample_lists(seed, ell, ids.shape[0], _ptr(ids), P, T, _ptr(out))
    return out


def priority(seed: int, ell: int, v: int) -> int:
    return int(lib().orc_priority(seed, ell, v))


def priorities(seed: int, ell: int, ids: np.ndarray) -> np.ndarray:
    return np.array([priority(seed, ell, int(v)) for v in ids], dtype=np.uint64)


def conflict_edges_allpairs(chars: np.ndarray, ids: np.ndarray, lists: np.ndarray, rel: int) -> np.ndarray:
    """Edges (a<b local indices) by the plain definition over all pairs."""
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    lists = np.ascontiguousarray(lists, dtype=np.uint32)
    q = chars.shape[1]
    m, T = lists.shape
    L = lib()
    cnt = L.orc_conflict_edges_allpairs(q, m, _ptr(ids), _ptr(chars), _ptr(lists), T, rel, None, 0)
    out = np.zeros((max(cnt, 1), 2), dtype=np.int32)
    L.orc_conflict_edges_allpairs(q, m, _ptr(ids), _ptr(chars), _ptr(lists), T, rel, _ptr(out), cnt)
    return out[:cnt]


def conflict_edges_bucketed(chars, ids, lists, P: int, rel: int, c_lo: int = 0, c_hi: int | None = None,
                            want_edges: bool = True):
    """Edges enumerated colour by colour (min-shared-colour rule).

    Returns (edges (k,2) int32 sorted, count, pair_tests)."""
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    lists = np.ascontiguousarray(lists, dtype=np.uint32)
    q = chars.shape[1]
    m, T = lists.shape
    if c_hi is None:
        c_hi = P
    tests = ctypes.c_int64()
    L = lib()
    if not want_edges:
        cnt = L.orc_conflict_edges_bucketed(q, m, _ptr(ids), _ptr(chars), _ptr(lists), T, P, rel, c_lo, c_hi,
                                            None, 0, ctypes.byref(tests))
        return None, cnt, tests.value
    # one pass sized by an upper bound would need C(m,2); count first instead
    cnt = L.orc_conflict_edges_bucketed(q, m, _ptr(ids), _ptr(chars), _ptr(lists), T, P, rel, c_lo, c_hi,
                                        None, 0, ctypes.byref(tests))
    if cnt < 0:
        raise MemoryError("oracle: allocation failed")
    out = np.zeros((max(cnt, 1), 2), dtype=np.int32)
    L.orc_conflict_edges_bucketed(q, m, _ptr(ids), _ptr(chars), _ptr(lists), T, P, rel, c_lo, c_hi,
                                  _ptr(out), cnt, ctypes.byref(tests))
    return out[:cnt], cnt, tests.value


def greedy_from_edges(prio: np.ndarray, lists: np.ndarray, P: int, edges: np.ndarray) -> np.ndarray:
    prio = np.ascontiguousarray(prio, dtype=np.uint64)
    lists = np.ascontiguousarray(lists, dtype=np.uint32)
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    m, T = lists.shape
    col = np.zeros(m, dtype=np.int32)
    rc = lib().orc_greedy_from_edges(m, _ptr(prio), _ptr(lists), T, P, _ptr(edges), edges.shape[0], _ptr(col))
    if rc != 0:
        raise MemoryError("oracle: allocation failed")
    return col


def greedy_dynamic(lists: np.ndarray, edges: np.ndarray, seed: int, ell: int):
    """Alg. 2 on a supplied graph.  Returns (colours[m] int32 with -1 for
    vertices whose list emptied, order[m]: vertices in the order taken)."""
    lists = np.ascontiguousarray(lists, dtype=np.uint32)
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    m, T = lists.shape
    col = np.zeros(max(m, 1), dtype=np.int32)
    order = np.zeros(max(m, 1), dtype=np.int32)
    rc = lib().orc_greedy_dynamic(m, _ptr(lists), T, _ptr(edges), edges.shape[0], seed, ell, _ptr(col), _ptr(order))
    if rc < 0:
        raise MemoryError("oracle: allocation failed")
    return col[:m], order[:m]


def greedy_dynamic_rounds(ids: np.ndarray, lists: np.ndarray, edges: np.ndarray, seed: int, ell: int,
                          divisor: int):
    """The round form of Alg. 2 on a supplied graph (ids: original ids, which
    key the draws).  Returns (colours[m] int32, -1 where the list emptied;
    rounds)."""
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    lists = np.ascontiguousarray(lists, dtype=np.uint32)
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    m, T = lists.shape
    col = np.zeros(max(m, 1), dtype=np.int32)
    nr = ctypes.c_int32()
    rc = lib().orc_greedy_dynamic_rounds(m, _ptr(ids), _ptr(lists), T, _ptr(edges), edges.shape[0], seed, ell,
                                         divisor, _ptr(col), ctypes.byref(nr))
    if rc < 0:
        raise MemoryError("oracle: allocation failed")
    return col[:m], nr.value


def color(x: np.ndarray, z: np.ndarray, q: int, seed: int, frac: float, alpha: float, rel: int,
          fixed_T: int = 0, max_stats: int = 4096, dynamic: bool = False, rounds_divisor: int = 0):
    """Full Picasso iteration.  Returns (n_colors, colors[n] int32, stats list).
    dynamic: colour each conflict graph by Alg. 2 instead of the static
    random order; rounds_divisor > 0 (with dynamic): by the round form of
    Alg. 2 with that divisor."""
    x = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, _words(q))
    z = np.ascontiguousarray(z, dtype=np.uint64).reshape(-1, _words(q))
    n = x.shape[0]
    out = np.zeros(max(n, 1), dtype=np.int32)
    stats = (IterStat * max_stats)()
    nit = ctypes.c_int32()
    if dynamic and rounds_divisor > 0:
        nc = lib().orc_color_dynamic_rounds(n, q, _ptr(x), _ptr(z), seed, frac, alpha, rel, fixed_T, rounds_divisor,
                                            _ptr(out), stats, max_stats, ctypes.byref(nit))
    else:
        fn = lib().orc_color_dynamic if dynamic else lib().orc_color
        nc = fn(n, q, _ptr(x), _ptr(z), seed, frac, alpha, rel, fixed_T, _ptr(out), stats, max_stats,
                ctypes.byref(nit))
    if nc < 0:
        raise MemoryError("oracle: allocation failed")
    st = [
        dict(m=s.m, P=s.P, T=s.T, pair_tests=s.pair_tests, edges=s.edges, colored=s.colored, offset=s.offset)
        for s in stats[: min(nit.value, max_stats)]
    ]
    return int(nc), out[:n], st


# ---- parameter schedule, features, predictor twin ---------------------------
MLP_IN, MLP_HIDDEN, MLP_OUT = 6, 64, 2
FEATURE_PAIRS = 4096


def _bind_extra():
    L = lib()
    if getattr(L, "_extra_bound", False):
        return L
    p = ctypes.c_void_p
    i32, i64, u32, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    L.orc_color_schedule.argtypes = [i64, i32, p, p, u64, p, p, i32, i32, p, p, i32, p]
    L.orc_color_schedule.restype = i64
    L.orc_features_bits.argtypes = [i64, i32, p, p, i64, p, u64, u32, i32, i32, p]
    L.orc_features_bits.restype = None
    L.orc_mlp_nparams.argtypes = []
    L.orc_mlp_nparams.restype = i32
    L.orc_mlp_forward.argtypes = [p, p, i32, p]
    L.orc_mlp_forward.restype = None
    L.orc_mlp_squash.argtypes = [p, p, p]
    L.orc_mlp_squash.restype = None
    L.orc_mlp_loss_grad.argtypes = [p, p, p, i32, p]
    L.orc_mlp_loss_grad.restype = dbl
    L.orc_adam_step.argtypes = [p, p, p, p, i32, dbl, dbl, dbl, dbl, i32]
    L.orc_adam_step.restype = None
    L.orc_count_conflict_edges.argtypes = [i32, i64, p, p, p, i32, i64, i32, i64, i64, p]
    L.orc_count_conflict_edges.restype = i64
    L.orc_greedy_by_classes.argtypes = [i32, i64, p, p, p, i32, i64, p, i32, p]
    L.orc_greedy_by_classes.restype = i32
    L.orc_color_classes.argtypes = [i64, i32, p, p, u64, p, p, i32, i32, i32, i32, p, p, i32, p]
    L.orc_color_classes.restype = i64
    L.orc_color_learned.argtypes = [i64, i32, p, p, u64, p, dbl, i32, i32, p, p, i32, p, p, i32]
    L.orc_color_learned.restype = i64
    L._extra_bound = True
    return L


def color_schedule(x, z, q, seed, fracs, alphas, rel, max_stats=4096):
    """Iteration l uses (fracs[l-1], alphas[l-1]), the last entry after the end."""
    L = _bind_extra()
    x = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, _words(q))
    z = np.ascontiguousarray(z, dtype=np.uint64).reshape(-1, _words(q))
    n = x.shape[0]
    fr = np.ascontiguousarray(fracs, dtype=np.float64)
    al = np.ascontiguousarray(alphas, dtype=np.float64)
    out = np.zeros(max(n, 1), dtype=np.int32)
    stats = (IterStat * max_stats)()
    nit = ctypes.c_int32()
    nc = L.orc_color_schedule(n, q, _ptr(x), _ptr(z), seed, _ptr(fr), _ptr(al), len(fr), rel, _ptr(out), stats,
                              max_stats, ctypes.byref(nit))
    if nc < 0:
        raise MemoryError("oracle: allocation failed")
    st = [dict(m=s.m, P=s.P, T=s.T, pair_tests=s.pair_tests, edges=s.edges, colored=s.colored, offset=s.offset)
          for s in stats[: min(nit.value, max_stats)]]
    return int(nc), out[:n], st


def features(x, z, q, ids, seed, ell, rel, K=FEATURE_PAIRS):
    L = _bind_extra()
    x = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, _words(q))
    z = np.ascontiguousarray(z, dtype=np.uint64).reshape(-1, _words(q))
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    out = np.zeros(5, dtype=np.float64)
    L.orc_features_bits(x.shape[0], q, _ptr(x), _ptr(z), ids.shape[0], _ptr(ids), seed, ell, rel, K, _ptr(out))
    return out


def mlp_nparams() -> int:
    return int(_bind_extra().orc_mlp_nparams())


def mlp_forward(params, raw):
    L = _bind_extra()
    params = np.ascontiguousarray(params, dtype=np.float64)
    raw = np.ascontiguousarray(raw, dtype=np.float64).reshape(-1, MLP_IN)
    out = np.zeros((raw.shape[0], MLP_OUT), dtype=np.float64)
    L.orc_mlp_forward(_ptr(params), _ptr(raw), raw.shape[0], _ptr(out))
    return out


def mlp_squash(o):
    L = _bind_extra()
    o = np.ascontiguousarray(o, dtype=np.float64)
    f, a = ctypes.c_double(), ctypes.c_double()
    L.orc_mlp_squash(_ptr(o), ctypes.byref(f), ctypes.byref(a))
    return f.value, a.value


def mlp_loss_grad(params, raw, target):
    L = _bind_extra()
    params = np.ascontiguousarray(params, dtype=np.float64)
    raw = np.ascontiguousarray(raw, dtype=np.float64).reshape(-1, MLP_IN)
    target = np.ascontiguousarray(target, dtype=np.float64).reshape(-1, MLP_OUT)
    grad = np.zeros_like(params)
    loss = L.orc_mlp_loss_grad(_ptr(params), _ptr(raw), _ptr(target), raw.shape[0], _ptr(grad))
    return loss, grad


def adam_step(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays params, m, v."""
    L = _bind_extra()
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, dtype=np.float64)
    L.orc_adam_step(_ptr(params), _ptr(g), _ptr(m), _ptr(v), step, lr, b1, b2, eps, params.shape[0])


# ---- runs without a stored conflict graph -----------------------------------

def _stats_list(stats, nit, max_stats):
    return [dict(m=s.m, P=s.P, T=s.T, pair_tests=s.pair_tests, edges=s.edges, colored=s.colored, offset=s.offset)
            for s in stats[: min(nit, max_stats)]]


def count_conflict_edges(chars, ids, lists, P: int, rel: int, c_lo: int = 0, c_hi: int | None = None):
    """|E_c| over the colour slice [c_lo, c_hi) without storing edges.
    Returns (count, pair_tests)."""
    L = _bind_extra()
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    lists = np.ascontiguousarray(lists, dtype=np.uint32)
    q = chars.shape[1]
    m, T = lists.shape
    tests = ctypes.c_int64()
    cnt = L.orc_count_conflict_edges(q, m, _ptr(ids), _ptr(chars), _ptr(lists), T, P, rel, c_lo,
                                     P if c_hi is None else c_hi, ctypes.byref(tests))
    if cnt < 0:
        raise MemoryError("oracle: allocation failed")
    return int(cnt), tests.value


def greedy_by_classes(chars, ids, lists, P: int, prio, rel: int) -> np.ndarray:
    """Static-order greedy of one iteration from the colour classes and the
    relation (no conflict graph)."""
    L = _bind_extra()
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    lists = np.ascontiguousarray(lists, dtype=np.uint32)
    prio = np.ascontiguousarray(prio, dtype=np.uint64)
    m, T = lists.shape
    col = np.zeros(max(m, 1), dtype=np.int32)
    if L.orc_greedy_by_classes(chars.shape[1], m, _ptr(ids), _ptr(chars), _ptr(lists), T, P, _ptr(prio), rel,
                               _ptr(col)):
        raise MemoryError("oracle: allocation failed")
    return col[:m]


def color_classes(x, z, q, seed, fracs, alphas, rel, fixed_T: int = 0, count_edges: bool = True,
                  max_stats: int = 4096):
    """Alg. 1 colouring each iteration from its colour classes (no stored
    conflict graph).  fracs/alphas: one value each (fixed parameters) or a
    per-iteration schedule.  Without count_edges the stats' edges are -1."""
    L = _bind_extra()
    x = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, _words(q))
    z = np.ascontiguousarray(z, dtype=np.uint64).reshape(-1, _words(q))
    n = x.shape[0]
    fr = np.ascontiguousarray(np.atleast_1d(fracs), dtype=np.float64)
    al = np.ascontiguousarray(np.atleast_1d(alphas), dtype=np.float64)
    out = np.zeros(max(n, 1), dtype=np.int32)
    stats = (IterStat * max_stats)()
    nit = ctypes.c_int32()
    nc = L.orc_color_classes(n, q, _ptr(x), _ptr(z), seed, _ptr(fr), _ptr(al), len(fr), rel, fixed_T,
                             int(count_edges), _ptr(out), stats, max_stats, ctypes.byref(nit))
    if nc < 0:
        raise MemoryError("oracle: allocation failed")
    return int(nc), out[:n], _stats_list(stats, nit.value, max_stats)


def color_learned(x, z, q, seed, params, rel, beta: float, count_edges: bool = True, max_stats: int = 4096):
    """Alg. 1 with each iteration's (f, alpha) from the FP64 predictor twin
    given the iteration's features and the trade-off weight beta.
    Returns (n_colors, colors, stats, schedule (iterations x 2 float64))."""
    L = _bind_extra()
    x = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, _words(q))
    z = np.ascontiguousarray(z, dtype=np.uint64).reshape(-1, _words(q))
    n = x.shape[0]
    params = np.ascontiguousarray(params, dtype=np.float64)
    assert params.shape == (mlp_nparams(),)
    out = np.zeros(max(n, 1), dtype=np.int32)
    stats = (IterStat * max_stats)()
    sched = np.zeros((max_stats, 2), dtype=np.float64)
    nit = ctypes.c_int32()
    nc = L.orc_color_learned(n, q, _ptr(x), _ptr(z), seed, _ptr(params), float(beta), rel, int(count_edges), _ptr(out), stats,
                             max_stats, ctypes.byref(nit), _ptr(sched), max_stats)
    if nc < 0:
        raise MemoryError("oracle: allocation failed")
    k = min(nit.value, max_stats)
    return int(nc), out[:n], _stats_list(stats, nit.value, max_stats), sched[:k].copy()
