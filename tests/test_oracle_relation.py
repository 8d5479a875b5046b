"""Pins for the oracle's pairwise relation (Sec. IV-A, Eq. 4-5; Sec. III).

Independent checks: explicit Kronecker products of the Pauli matrices of
Eq. 4, per-qubit 2x2 commutators for qubit-wise commutativity, the paper's
3-bit "inverse one-hot" code (Sec. IV-A), and textbook special cases.
"""
import itertools

import numpy as np
import pytest

from paper_2401_06713_amd import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore")

SIGMA = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def kron_string(s):
    m = np.eye(1, dtype=complex)
    for ch in s:
        m = np.kron(m, SIGMA[ch])
    return m


def encode(strings, q):
    """chars -> bit planes, written from the layout definition."""
    W = wl.words(q)
    x = np.zeros((len(strings), W), np.uint64)
    z = np.zeros((len(strings), W), np.uint64)
    for i, s in enumerate(strings):
        for k, ch in enumerate(s):
            b = np.uint64(1) << np.uint64(k % 64)
            if ch in "XY":
                x[i, k // 64] |= b
            if ch in "YZ":
                z[i, k // 64] |= b
    return x, z


def test_decode_roundtrip(orc):
    rng = np.random.default_rng(1)
    for q in (1, 5, 63, 64, 65, 130):
        strings = ["".join(rng.choice(list("IXYZ"), size=q)) for _ in range(20)]
        x, z = encode(strings, q)
        dec = orc.decode(x, z, q)
        assert [bytes(r).decode() for r in dec] == strings


def test_single_qubit_rule_matches_matrices(orc):
    # Eq. 5: distinct non-identity Pauli matrices anticommute; all others commute.
    for a, b in itertools.product("IXYZ", repeat=2):
        A, B = SIGMA[a], SIGMA[b]
        anti = np.allclose(A @ B + B @ A, 0)
        comm = np.allclose(A @ B - B @ A, 0)
        assert anti != comm  # exactly one holds
        assert orc.qubit_anticommutes(a, b) == anti


def test_three_bit_code(orc):
    # Sec. IV-A: X=110, Y=101, Z=011, I=000; the LSB of popcount(AND) flags a mismatch.
    enc = {"I": 0b000, "X": 0b110, "Y": 0b101, "Z": 0b011}
    for a, b in itertools.product("IXYZ", repeat=2):
        assert (bin(enc[a] & enc[b]).count("1") & 1) == int(orc.qubit_anticommutes(a, b))


@pytest.mark.parametrize("q", [1, 2, 3])
def test_anticommute_all_pairs_vs_kronecker(orc, q):
    strings = ["".join(p) for p in itertools.product("IXYZ", repeat=q)]
    mats = {s: kron_string(s) for s in strings}
    for a in strings:
        for b in strings:
            A, B = mats[a], mats[b]
            anti = np.allclose(A @ B + B @ A, 0)
            comm = np.allclose(A @ B - B @ A, 0)
            assert anti != comm
            assert orc.relation_chars(a.encode(), b.encode(), 0) == anti


@pytest.mark.parametrize("q", [1, 2, 3])
def test_commute_all_pairs_vs_kronecker(orc, q):
    # COMMUTE (the paper's own orientation): an edge iff the matrices commute
    strings = ["".join(p) for p in itertools.product("IXYZ", repeat=q)]
    mats = {s: kron_string(s) for s in strings}
    for a in strings:
        for b in strings:
            A, B = mats[a], mats[b]
            assert orc.relation_chars(a.encode(), b.encode(), 2) == np.allclose(A @ B - B @ A, 0)


def test_anticommute_random_q4_vs_kronecker(orc):
    rng = np.random.default_rng(7)
    for _ in range(300):
        a = "".join(rng.choice(list("IXYZ"), 4))
        b = "".join(rng.choice(list("IXYZ"), 4))
        A, B = kron_string(a), kron_string(b)
        assert orc.relation_chars(a.encode(), b.encode(), 0) == np.allclose(A @ B + B @ A, 0)


@pytest.mark.parametrize("q", [1, 2, 3, 6])
def test_qwc_vs_per_qubit_commutators(orc, q):
    rng = np.random.default_rng(q)
    for _ in range(400):
        a = "".join(rng.choice(list("IXYZ"), q))
        b = "".join(rng.choice(list("IXYZ"), q))
        qwc = all(np.allclose(SIGMA[s] @ SIGMA[t], SIGMA[t] @ SIGMA[s]) for s, t in zip(a, b))
        assert orc.relation_chars(a.encode(), b.encode(), 1) == (not qwc)


def test_qwc_implies_commute(orc):
    # Qubit-wise commuting strings commute; so "anticommute" implies "not QWC".
    rng = np.random.default_rng(3)
    for _ in range(2000):
        a = "".join(rng.choice(list("IXYZ"), 5)).encode()
        b = "".join(rng.choice(list("IXYZ"), 5)).encode()
        if orc.relation_chars(a, b, 0):
            assert orc.relation_chars(a, b, 1)


@pytest.mark.parametrize("q", [3, 8, 70])
def test_majorana_strings_pairwise_anticommute(orc, q):
    x, z = wl.majorana_strings(q)
    ch = orc.decode(x, z, q)
    n = ch.shape[0]
    for i in range(n):
        for j in range(n):
            r = orc.relation_chars(ch[i].tobytes(), ch[j].tobytes(), 0)
            assert r == (i != j)
    if q <= 8:  # and the matrices agree
        mats = [kron_string(bytes(r).decode()) for r in ch]
        for i in range(n):
            for j in range(i + 1, n):
                assert np.allclose(mats[i] @ mats[j] + mats[j] @ mats[i], 0)


def test_iz_strings_commute_and_qwc(orc):
    x, z = wl.iz_strings(40, 12, seed=5)
    ch = orc.decode(x, z, 12)
    for i in range(40):
        for j in range(40):
            assert not orc.relation_chars(ch[i].tobytes(), ch[j].tobytes(), 0)
            assert not orc.relation_chars(ch[i].tobytes(), ch[j].tobytes(), 1)


def test_disjoint_supports_are_qwc(orc):
    rng = np.random.default_rng(11)
    for _ in range(200):
        q = 10
        a = ["I"] * q
        b = ["I"] * q
        for k in range(q):
            r = rng.integers(3)
            if r == 0:
                a[k] = rng.choice(list("XYZ"))
            elif r == 1:
                b[k] = rng.choice(list("XYZ"))
        A, B = "".join(a).encode(), "".join(b).encode()
        assert not orc.relation_chars(A, B, 1)
        assert not orc.relation_chars(A, B, 0)
