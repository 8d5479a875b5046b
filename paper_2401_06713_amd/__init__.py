"""MI355X palette colouring of Pauli strings (Picasso, arXiv 2401.06713).

Thin ctypes binding over libpicasso.so (include/picasso.h): argument
marshalling only.  Every step of the method runs in the library's HIP
kernels; there is no CPU fallback, and loading fails loudly when the built
library is missing.  PyTorch tensors are accepted wherever the C ABI takes
device pointers (torch is used for device memory and streams only).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpicasso.so")

REL_ANTICOMMUTE = 0
REL_QWC = 1
REL_COMMUTE = 2
PATH_AUTO, PATH_VALU, PATH_MFMA = 0, 1, 2
(OPT_MEM_BUDGET, OPT_PAIR_PATH, OPT_FIXED_T, OPT_STREAM, OPT_TIMING, OPT_JP_BATCH, OPT_GRAPH,
 OPT_MFMA_CAP, OPT_TAIL, OPT_LEARNED_JUDGE, OPT_CSR_SIZING, OPT_COLOURER, OPT_DYN_DIVISOR, OPT_EDGES,
 OPT_BUCKET_BUILD) = range(1, 16)
COLOURER_STATIC, COLOURER_DYNAMIC = 0, 1
JUDGE_NONE, JUDGE_LEARNED, JUDGE_FIXED = 0, 1, 2
MAX_T = 1024
MAX_ITER_STATS = 256

EINVAL, ENOMEM, EDEVICE, EINTERNAL = -1, -2, -3, -4

# Every entry point declared in include/picasso.h.
EXPORTS = (
    "picasso_last_error",
    "picasso_create",
    "picasso_create_device",
    "picasso_create_batch",
    "picasso_destroy",
    "picasso_set_option",
    "picasso_color",
    "picasso_color_device",
    "picasso_color_batch",
    "picasso_color_batch_device",
    "picasso_get_stats",
    "picasso_get_instance_stats",
    "picasso_sample_lists",
    "picasso_conflict_graph",
    "picasso_list_color_csr",
    "picasso_features",
    "picasso_mlp_create",
    "picasso_mlp_destroy",
    "picasso_mlp_get_params",
    "picasso_mlp_set_params",
    "picasso_mlp_forward",
    "picasso_mlp_gradient",
    "picasso_mlp_train_step",
    "picasso_color_schedule",
    "picasso_color_learned",
    "picasso_color_device_noalloc",
)
MLP_NPARAMS = 4738
MLP_INPUTS = 6
FEATURE_PAIRS = 4096


class IterStats(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("P", ctypes.c_int64),
        ("T", ctypes.c_int64),
        ("pair_tests", ctypes.c_int64),
        ("edges", ctypes.c_int64),
        ("edges_bound", ctypes.c_int64),
        ("colored", ctypes.c_int64),
        ("offset", ctypes.c_int64),
        ("pair_path", ctypes.c_int32),
        ("jp_rounds", ctypes.c_int32),
        ("ms_graph", ctypes.c_double),
        ("ms_buckets", ctypes.c_double),
        ("ms_count", ctypes.c_double),
        ("ms_fill", ctypes.c_double),
        ("ms_color", ctypes.c_double),
        ("ms_compact", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("n_colors", ctypes.c_int64),
        ("palette_total", ctypes.c_int64),
        ("pair_tests", ctypes.c_int64),
        ("edges", ctypes.c_int64),
        ("max_edges", ctypes.c_int64),
        ("peak_device_bytes", ctypes.c_int64),
        ("n_iters", ctypes.c_int32),
        ("judged", ctypes.c_int32),
        ("csr_refills", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("ms_total", ctypes.c_double),
        ("iters", IterStats * MAX_ITER_STATS),
    ]

    def to_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("iters", "reserved")}
        d["iters"] = [
            {k: getattr(it, k) for k, _ in IterStats._fields_}
            for it in self.iters[: min(self.n_iters, MAX_ITER_STATS)]
        ]
        return d


class InstanceStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("n_colors", ctypes.c_int64),
        ("palette_total", ctypes.c_int64),
        ("edges", ctypes.c_int64),
        ("max_edges", ctypes.c_int64),
        ("n_iters", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class PicassoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"picasso error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libpicasso.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2401_06713_amd.build_lib` "
            "(the HIP library is required; there is no fallback)"
        )
    # One HIP runtime per process: torch ships its own libamdhip64.so.7.  If it
    # is imported first, the library's dependency resolves to that same copy;
    # loaded the other way round, torch would bring a second runtime that
    # cannot initialise the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    p, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    L.picasso_last_error.restype = ctypes.c_char_p
    L.picasso_last_error.argtypes = []
    L.picasso_create.restype = p
    L.picasso_create.argtypes = [i64, i32, p, p]
    L.picasso_create_device.restype = p
    L.picasso_create_device.argtypes = [i64, i32, p, p]
    L.picasso_create_batch.restype = p
    L.picasso_create_batch.argtypes = [i32, p, p, p, p]
    L.picasso_color_batch.restype = i64
    L.picasso_color_batch.argtypes = [p, p, p, p, p, p, p]
    L.picasso_color_batch_device.restype = i64
    L.picasso_color_batch_device.argtypes = [p, p, p, p, p, p, p]
    L.picasso_get_instance_stats.restype = i32
    L.picasso_get_instance_stats.argtypes = [p, i32, p]
    L.picasso_destroy.restype = None
    L.picasso_destroy.argtypes = [p]
    L.picasso_set_option.restype = i32
    L.picasso_set_option.argtypes = [p, i32, i64]
    L.picasso_color.restype = i64
    L.picasso_color.argtypes = [p, u64, dbl, dbl, i32, p]
    L.picasso_color_device.restype = i64
    L.picasso_color_device.argtypes = [p, u64, dbl, dbl, i32, p]
    L.picasso_get_stats.restype = i32
    L.picasso_get_stats.argtypes = [p, ctypes.POINTER(Stats)]
    L.picasso_sample_lists.restype = i32
    L.picasso_sample_lists.argtypes = [p, u64, i32, i64, p, i64, i32, p, p]
    L.picasso_conflict_graph.restype = i64
    L.picasso_conflict_graph.argtypes = [p, u64, i32, i64, p, i64, i32, i32, p, p, i64]
    L.picasso_list_color_csr.restype = i64
    L.picasso_list_color_csr.argtypes = [p, i64, p, p, i32, i64, p, p, p]
    f32 = ctypes.c_float
    L.picasso_features.restype = i32
    L.picasso_features.argtypes = [p, u64, i32, i64, p, i32, p]
    L.picasso_mlp_create.restype = p
    L.picasso_mlp_create.argtypes = [p, u64]
    L.picasso_mlp_destroy.restype = None
    L.picasso_mlp_destroy.argtypes = [p]
    L.picasso_mlp_get_params.restype = i32
    L.picasso_mlp_get_params.argtypes = [p, p]
    L.picasso_mlp_set_params.restype = i32
    L.picasso_mlp_set_params.argtypes = [p, p]
    L.picasso_mlp_forward.restype = i32
    L.picasso_mlp_forward.argtypes = [p, p, i32, p]
    L.picasso_mlp_gradient.restype = i32
    L.picasso_mlp_gradient.argtypes = [p, p, p, i32, p, ctypes.POINTER(f32)]
    L.picasso_mlp_train_step.restype = i32
    L.picasso_mlp_train_step.argtypes = [p, p, p, i32, f32, ctypes.POINTER(f32)]
    L.picasso_color_schedule.restype = i64
    L.picasso_color_schedule.argtypes = [p, u64, p, p, i32, i32, p]
    L.picasso_color_learned.restype = i64
    L.picasso_color_learned.argtypes = [p, u64, p, dbl, i32, p, p, i32]
    L.picasso_color_device_noalloc.restype = i64
    L.picasso_color_device_noalloc.argtypes = [i64, i32, p, p, u64, dbl, dbl, i32, p, p]
    _lib = L
    return L


def last_error() -> str:
    return lib().picasso_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise PicassoError(rc, last_error())
    return rc


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _is_tensor(a) -> bool:
    return type(a).__module__.startswith("torch")


class Picasso:
    """A set of n Pauli strings on q qubits held on the device.

    x, z: (n, W) uint64 host arrays (numpy), or device tensors (torch,
    int64/uint64 on cuda) -- the latter are copied device-to-device.
    """

    def __init__(self, x, z, q: int):
        L = lib()
        self.q = int(q)
        self.W = (self.q + 63) // 64
        if _is_tensor(x):
            assert x.is_cuda and z.is_cuda and x.is_contiguous() and z.is_contiguous()
            self.n = int(x.shape[0])
            h = L.picasso_create_device(self.n, self.q, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(z.data_ptr()))
        else:
            x = np.ascontiguousarray(x, dtype=np.uint64)
            z = np.ascontiguousarray(z, dtype=np.uint64)
            self.n = int(x.shape[0])
            if x.shape != z.shape or (self.W > 0 and x.size != self.n * self.W):
                raise PicassoError(EINVAL, f"x/z must both be (n, {self.W}) uint64")
            h = L.picasso_create(self.n, self.q, _ptr(x), _ptr(z))
        if not h:
            raise PicassoError(EINVAL, last_error())
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().picasso_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_option(self, key: int, value: int):
        _check(lib().picasso_set_option(self._h, key, int(value)))

    def color(self, seed: int = 0, palette_frac: float = 0.125, list_size: float = 2.0,
              relation: int = REL_ANTICOMMUTE):
        """Returns (n_colors, colors int32[n]) with colours on the host."""
        out = np.empty(max(self.n, 1), dtype=np.int32)
        nc = _check(lib().picasso_color(self._h, seed, palette_frac, list_size, relation, _ptr(out)))
        return nc, out[: self.n]

    def color_device(self, out, seed: int = 0, palette_frac: float = 0.125, list_size: float = 2.0,
                     relation: int = REL_ANTICOMMUTE) -> int:
        """Colours into a device int32 tensor `out` of n entries; returns n_colors."""
        assert out.is_cuda and out.numel() >= self.n
        return _check(lib().picasso_color_device(self._h, seed, palette_frac, list_size, relation,
                                                 ctypes.c_void_p(out.data_ptr())))

    def stats(self) -> dict:
        s = Stats()
        _check(lib().picasso_get_stats(self._h, ctypes.byref(s)))
        return s.to_dict()

    def instance_stats(self) -> list[dict]:
        nb = _check(lib().picasso_get_instance_stats(self._h, 0, None))
        arr = (InstanceStats * nb)()
        _check(lib().picasso_get_instance_stats(self._h, nb, arr))
        return [{k: getattr(r, k) for k, _ in InstanceStats._fields_ if k != "reserved"} for r in arr]

    def sample_lists(self, seed: int, ell: int, ids, P: int, T: int):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        m = ids.shape[0]
        lists = np.zeros((max(m, 1), T), dtype=np.uint32)
        prio = np.zeros(max(m, 1), dtype=np.uint64)
        _check(lib().picasso_sample_lists(self._h, seed, ell, m, _ptr(ids), P, T, _ptr(lists), _ptr(prio)))
        return lists[:m], prio[:m]

    def conflict_graph(self, seed: int, ell: int, ids, P: int, T: int, relation: int):
        """Returns (rowptr int64[m+1], adj int32[2|E|]) -- rows unordered."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        m = ids.shape[0]
        rowptr = np.zeros(m + 1, dtype=np.int64)
        L = lib()
        ne = _check(L.picasso_conflict_graph(self._h, seed, ell, m, _ptr(ids), P, T, relation, _ptr(rowptr), None, 0))
        adj = np.zeros(max(2 * ne, 1), dtype=np.int32)
        ne2 = _check(L.picasso_conflict_graph(self._h, seed, ell, m, _ptr(ids), P, T, relation, _ptr(rowptr),
                                              _ptr(adj), adj.shape[0]))
        assert ne2 == ne
        return rowptr, adj[: 2 * ne]


    def conflict_rowptr(self, seed: int, ell: int, ids, P: int, T: int, relation: int):
        """Returns (|E_c|, rowptr int64[m+1]): the CSR row pointers (vertex
        degrees) without copying the adjacency to the host."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        m = ids.shape[0]
        rowptr = np.zeros(m + 1, dtype=np.int64)
        ne = _check(lib().picasso_conflict_graph(self._h, seed, ell, m, _ptr(ids), P, T, relation, _ptr(rowptr),
                                                 None, 0))
        return ne, rowptr

    def features(self, seed: int, ell: int, ids, relation: int) -> np.ndarray:
        """(ln m, q, mean Pauli weight, sampled relation density, ell)."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        out = np.zeros(5, dtype=np.float64)
        _check(lib().picasso_features(self._h, seed, ell, ids.shape[0], _ptr(ids), relation, _ptr(out)))
        return out

    def color_schedule(self, seed: int, palette_fracs, list_sizes, relation: int = REL_ANTICOMMUTE):
        """Colours with iteration l using entry min(l, len) - 1 of the
        schedule; returns (n_colors, colors int32[n])."""
        fr = np.ascontiguousarray(np.atleast_1d(palette_fracs), dtype=np.float64)
        al = np.ascontiguousarray(np.atleast_1d(list_sizes), dtype=np.float64)
        if fr.shape != al.shape:
            raise PicassoError(EINVAL, "schedule arrays differ in length")
        out = np.empty(max(self.n, 1), dtype=np.int32)
        nc = _check(lib().picasso_color_schedule(self._h, seed, _ptr(fr), _ptr(al), fr.shape[0], relation,
                                                 _ptr(out)))
        return nc, out[: self.n]

    def color_learned(self, mlp: "Mlp", seed: int = 0, relation: int = REL_ANTICOMMUTE, beta: float = 0.5,
                      max_sched: int = 256):
        """Colours with per-iteration (f, alpha) from the network given the
        iteration's features and beta.

        Returns (n_colors, colors, schedule) with schedule (iterations, 2) float32."""
        out = np.empty(max(self.n, 1), dtype=np.int32)
        sched = np.zeros((max_sched, 2), dtype=np.float32)
        nc = _check(lib().picasso_color_learned(self._h, seed, mlp._m, beta, relation, _ptr(out), _ptr(sched),
                                                max_sched))
        n_it = min(self.stats()["n_iters"], max_sched)
        return nc, out[: self.n], sched[:n_it].copy()


class PicassoBatch(Picasso):
    """Many independent instances in one handle, coloured together.

    instances: sequence of (x, z, q) with x, z (n_i, ceil(q_i/64)) uint64
    host arrays.  Only color_batch, stats and instance_stats apply (the
    single-instance calls reject a handle of more than one instance).
    """

    def __init__(self, instances):
        L = lib()
        xs, zs, ns, qs = [], [], [], []
        for x, z, q in instances:
            x = np.ascontiguousarray(x, dtype=np.uint64)
            z = np.ascontiguousarray(z, dtype=np.uint64)
            W = (int(q) + 63) // 64
            if x.shape != z.shape or x.size != x.shape[0] * W:
                raise PicassoError(EINVAL, f"x/z must both be (n, {W}) uint64")
            xs.append(x.reshape(-1))
            zs.append(z.reshape(-1))
            ns.append(x.shape[0])
            qs.append(int(q))
        self.count = len(ns)
        self.ns = np.asarray(ns, dtype=np.int64)
        self.qs = np.asarray(qs, dtype=np.int32)
        self.offsets = np.concatenate([[0], np.cumsum(self.ns)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        self.q = int(self.qs.max()) if self.count else 0
        self.W = (self.q + 63) // 64
        xc = np.concatenate(xs) if xs else np.zeros(0, np.uint64)
        zc = np.concatenate(zs) if zs else np.zeros(0, np.uint64)
        xc = np.ascontiguousarray(xc if xc.size else np.zeros(1, np.uint64))
        zc = np.ascontiguousarray(zc if zc.size else np.zeros(1, np.uint64))
        h = L.picasso_create_batch(self.count, _ptr(self.ns) if self.count else None,
                                   _ptr(self.qs) if self.count else None, _ptr(xc), _ptr(zc))
        if not h:
            raise PicassoError(EINVAL, last_error())
        self._h = ctypes.c_void_p(h)

    def color_batch(self, seeds, palette_fracs, list_sizes, relations):
        """Returns (n_colors int64[count], [colors int32[n_i] per instance])."""
        k = self.count
        seeds, fr, al, rel = self._batch_args(seeds, palette_fracs, list_sizes, relations)
        out = np.empty(max(self.n, 1), dtype=np.int32)
        nc = np.zeros(max(k, 1), dtype=np.int64)
        _check(lib().picasso_color_batch(self._h, _ptr(seeds), _ptr(fr), _ptr(al), _ptr(rel), _ptr(out), _ptr(nc)))
        cols = [out[self.offsets[i]:self.offsets[i + 1]].copy() for i in range(k)]
        return nc[:k], cols

    def color_batch_device(self, out, seeds, palette_fracs, list_sizes, relations):
        """Colours into a device int32 tensor `out` (total strings); returns
        n_colors int64[count] (instance i's colours at out[offsets[i]:offsets[i+1]])."""
        assert out.is_cuda and out.numel() >= self.n
        k = self.count
        args = self._batch_args(seeds, palette_fracs, list_sizes, relations)
        nc = np.zeros(max(k, 1), dtype=np.int64)
        _check(lib().picasso_color_batch_device(self._h, *map(_ptr, args), ctypes.c_void_p(out.data_ptr()), _ptr(nc)))
        return nc[:k]

    def _batch_args(self, seeds, palette_fracs, list_sizes, relations):
        k = self.count
        return (np.ascontiguousarray(np.broadcast_to(np.asarray(seeds, dtype=np.uint64), (k,))),
                np.ascontiguousarray(np.broadcast_to(np.asarray(palette_fracs, dtype=np.float64), (k,))),
                np.ascontiguousarray(np.broadcast_to(np.asarray(list_sizes, dtype=np.float64), (k,))),
                np.ascontiguousarray(np.broadcast_to(np.asarray(relations, dtype=np.int32), (k,))))


class Mlp:
    """The 5 -> 64 -> 64 -> 2 parameter predictor on the device (FP32)."""

    def __init__(self, params=None, seed: int = 0):
        L = lib()
        if params is not None:
            params = np.ascontiguousarray(params, dtype=np.float32)
            assert params.shape == (MLP_NPARAMS,)
        m = L.picasso_mlp_create(_ptr(params) if params is not None else None, seed)
        if not m:
            raise PicassoError(EINVAL, last_error())
        self._m = ctypes.c_void_p(m)

    def close(self):
        if getattr(self, "_m", None):
            lib().picasso_mlp_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def get_params(self) -> np.ndarray:
        out = np.zeros(MLP_NPARAMS, dtype=np.float32)
        _check(lib().picasso_mlp_get_params(self._m, _ptr(out)))
        return out

    def set_params(self, params):
        params = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().picasso_mlp_set_params(self._m, _ptr(params)))

    def forward(self, feats) -> np.ndarray:
        feats = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, MLP_INPUTS)
        out = np.zeros((feats.shape[0], 2), dtype=np.float32)
        _check(lib().picasso_mlp_forward(self._m, _ptr(feats), feats.shape[0], _ptr(out)))
        return out

    def gradient(self, feats, target):
        feats = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, MLP_INPUTS)
        target = np.ascontiguousarray(target, dtype=np.float32).reshape(-1, 2)
        grad = np.zeros(MLP_NPARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        _check(lib().picasso_mlp_gradient(self._m, _ptr(feats), _ptr(target), feats.shape[0], _ptr(grad),
                                          ctypes.byref(loss)))
        return loss.value, grad

    def train_step(self, feats, target, lr: float = 1e-3) -> float:
        feats = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, MLP_INPUTS)
        target = np.ascontiguousarray(target, dtype=np.float32).reshape(-1, 2)
        loss = ctypes.c_float()
        _check(lib().picasso_mlp_train_step(self._m, _ptr(feats), _ptr(target), feats.shape[0], lr,
                                            ctypes.byref(loss)))
        return loss.value


def list_color_csr(prio, lists, P: int, rowptr, adj, handle: Picasso | None = None):
    """Jones-Plassmann list colouring of a given symmetric CSR."""
    prio = np.ascontiguousarray(prio, dtype=np.uint64)
    lists = np.ascontiguousarray(lists, dtype=np.uint32)
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    m, T = lists.shape
    own = handle is None
    if own:
        handle = Picasso(np.zeros((1, 1), np.uint64), np.ones((1, 1), np.uint64), 1)
    try:
        col = np.zeros(max(m, 1), dtype=np.int32)
        _check(lib().picasso_list_color_csr(handle._h, m, _ptr(prio), _ptr(lists), T, P, _ptr(rowptr),
                                            _ptr(adj) if adj.size else None, _ptr(col)))
        return col[:m]
    finally:
        if own:
            handle.close()


def edges_from_csr(rowptr: np.ndarray, adj: np.ndarray) -> np.ndarray:
    """Canonical sorted (a<b) edge list from a symmetric CSR."""
    m = rowptr.shape[0] - 1
    src = np.repeat(np.arange(m, dtype=np.int64), np.diff(rowptr))
    dst = adj.astype(np.int64)
    keep = src < dst
    key = np.sort(src[keep] * (1 << 32) + dst[keep])
    return np.stack([key >> 32, key & 0xFFFFFFFF], axis=1).astype(np.int32)
