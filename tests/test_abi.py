"""The C ABI library loads on a CPU-only host and exports every entry point
that include/picasso.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import paper_2401_06713_amd as pk

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "picasso.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(picasso_[a-z_]+)\s*\(", text)))


def test_header_matches_binding():
    assert declared_functions() == sorted(pk.EXPORTS)


def test_library_exports_every_symbol():
    L = ctypes.CDLL(pk.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_last_error_callable_without_gpu():
    assert isinstance(pk.last_error(), str)


def test_stats_struct_layout():
    # picasso_iter_stats: 7 int64 + 2 int32 + 6 double = 112 bytes
    assert ctypes.sizeof(pk.IterStats) == 112
    assert ctypes.sizeof(pk.Stats) == 7 * 8 + 8 + 8 + 112 * pk.MAX_ITER_STATS


def test_instance_stats_struct_layout():
    # picasso_instance_stats: 5 int64 + 2 int32 = 48 bytes
    assert ctypes.sizeof(pk.InstanceStats) == 48
