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


def c_layout(struct: str, fields) -> dict:
    """sizeof and offsetof of a header struct, from the C compiler."""
    import subprocess
    import tempfile

    body = [f'printf("size %zu\\n", sizeof({struct}));']
    body += [f'printf("{f} %zu\\n", offsetof({struct}, {f}));' for f in fields]
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"picasso.h\"\nint main(void) {\n"
           + "\n".join(body) + "\nreturn 0;\n}\n")
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(c, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (line.split() for line in out.splitlines())}


def check_struct(struct: str, cls):
    names = [name for name, _ in cls._fields_]
    lay = c_layout(struct, names)
    assert ctypes.sizeof(cls) == lay["size"], struct
    for name in names:
        assert getattr(cls, name).offset == lay[name], (struct, name)


def test_stats_struct_layout():
    check_struct("picasso_iter_stats", pk.IterStats)
    check_struct("picasso_stats", pk.Stats)


def test_instance_stats_struct_layout():
    check_struct("picasso_instance_stats", pk.InstanceStats)
