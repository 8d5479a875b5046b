"""picasso_color_device_noalloc (the colouring with all working memory in a
fixed device array) against picasso_color_device on a handle of the same
strings: bit-exact colours and equal colour counts, on two calls in a row
with the second instance smaller than the first, for every relation; sizes
beyond the stated maximum are rejected."""
import ctypes
import sys

import numpy as np
import pytest

import paper_2401_06713_amd as pk
from paper_2401_06713_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def noalloc(xd, zd, q, seed, f, a, rel, out):
    import torch

    n = int(xd.shape[0])
    stream = torch.cuda.current_stream().cuda_stream
    rc = pk.lib().picasso_color_device_noalloc(n, q, ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(zd.data_ptr()),
                                               seed, f, a, rel, ctypes.c_void_p(out.data_ptr()),
                                               ctypes.c_void_p(stream))
    return rc


def reference(x, z, q, seed, f, a, rel):
    import torch

    n = x.shape[0]
    out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    with pk.Picasso(x, z, q) as h:
        nc = h.color_device(out, seed, f, a, rel)
    return nc, out.cpu().numpy()


@pytest.mark.parametrize("rel", [pk.REL_ANTICOMMUTE, pk.REL_QWC, pk.REL_COMMUTE])
def test_noalloc_matches_color_device(rel):
    import torch

    torch.cuda.set_device(0)
    cases = [(256, 70, 0.7, 11, 0.125, 2.0), (97, 130, 0.5, 12, 0.3, 1.5)]  # second call smaller
    for n, q, pI, seed, f, a in cases:
        say("noalloc", rel, n, q, seed, f, a)
        r = (1 - pI) / 3
        x, z = wl.pauli_strings(n, q, (pI, r, r, r), seed=seed)
        xd = torch.from_numpy(x.view(np.int64)).cuda()
        zd = torch.from_numpy(z.view(np.int64)).cuda()
        out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        nc = noalloc(xd, zd, q, seed, f, a, rel, out)
        torch.cuda.synchronize()
        assert nc >= 0, pk.last_error()
        rnc, rcol = reference(x, z, q, seed, f, a, rel)
        col = out.cpu().numpy()
        assert nc == rnc
        assert np.array_equal(col, rcol)
        assert (col >= 0).all() and np.unique(col).size == nc


def test_noalloc_rejects_beyond_maximum():
    import torch

    torch.cuda.set_device(0)
    q = 20
    x, z = wl.pauli_strings(257, q, seed=3)
    xd = torch.from_numpy(x.view(np.int64)).cuda()
    zd = torch.from_numpy(z.view(np.int64)).cuda()
    out = torch.full((257,), -7, dtype=torch.int32, device="cuda")
    assert noalloc(xd, zd, q, 0, 0.125, 2.0, 0, out) == pk.EINVAL
    assert "at most 256" in pk.last_error()
    # lists that exceed the kernel's list entries: T = P = m for f = 1, alpha = 30
    assert noalloc(xd[:200], zd[:200], q, 0, 1.0, 30.0, 0, out) == pk.EINVAL
    assert "list entries" in pk.last_error()
    # padding bits above q
    xb = xd[:10].clone()
    xb[3] |= 1 << 40
    assert noalloc(xb, zd[:10], q, 0, 0.125, 2.0, 0, out) == pk.EINVAL
    assert (out == -7).all().item()
