"""Pins for the oracle's parameters, lists and priorities.

Parameters (Alg. 1 estimate step, Table I, Sec. VII): the configuration sizes
printed with the workloads fix the natural log and the ceilings.
Lists (Sec. IV: T colours uniformly at random from the palette) are pinned
by structure and by statistics; the Philox4x32-10 generator under them by its
authors' published known-answer vectors (tests/golden/philox4x32_10_kat.txt).
"""
import math
import os

import numpy as np
import pytest
from scipy import stats


def test_params_printed_values(orc):
    # n=2000: P = ceil(0.125 n) = 250 and T = ceil(2 ln n) = 16 as printed.
    assert orc.params(2000, 0.125, 2.0) == (250, 16)
    assert orc.params(200_000, 0.125, 2.0) == (25_000, 25)
    assert orc.params(2_000_000, 0.125, 2.0) == (250_000, 30)
    assert orc.params(500_000, 0.125, 2.0) == (62_500, 27)
    # log2 would give 22, log10 would give 7
    assert orc.params(2000, 0.125, 2.0)[1] == math.ceil(2 * math.log(2000))


def test_params_clamps(orc):
    assert orc.params(1, 0.125, 2.0) == (1, 1)  # ln 1 = 0 -> T = 1
    assert orc.params(2, 0.125, 2.0) == (1, 1)  # P = 1 caps T
    assert orc.params(10, 1.0, 100.0) == (10, 10)
    assert orc.params(1000, 0.5, 2.0, fixed_T=7) == (500, 7)
    assert orc.params(3, 0.5, 2.0, fixed_T=7) == (2, 2)


@pytest.mark.parametrize("P,T", [(1, 1), (5, 2), (50, 10), (250, 16), (25_000, 25), (10, 10), (3000, 256)])
def test_list_structure(orc, P, T):
    for v in range(40):
        L = orc.sample_list(123, 1, v, P, T)
        assert L.shape == (T,)
        assert np.all(np.diff(L.astype(np.int64)) > 0)  # sorted, distinct
        assert L[0] >= 0 and L[-1] < P


def test_full_palette_when_T_equals_P(orc):
    for v in range(10):
        assert np.array_equal(orc.sample_list(9, 2, v, 17, 17), np.arange(17, dtype=np.uint32))


def test_colour_marginals_uniform(orc):
    P, T, m = 50, 10, 20000
    lists = orc.sample_lists(5, 1, np.arange(m, dtype=np.int32), P, T)
    counts = np.bincount(lists.ravel(), minlength=P)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4, (chi2, p)


def test_subsets_uniform(orc):
    # every T-subset equally likely (catches a biased Floyd step)
    P, T, m = 6, 3, 30000
    lists = orc.sample_lists(17, 3, np.arange(m, dtype=np.int32), P, T)
    keys = lists[:, 0] * 36 + lists[:, 1] * 6 + lists[:, 2]
    _, counts = np.unique(keys, return_counts=True)
    assert counts.size == math.comb(P, T)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4, (chi2, p)


def test_pair_share_probability(orc):
    P, T, m = 200, 12, 6000
    a = orc.sample_lists(1, 1, np.arange(m, dtype=np.int32), P, T)
    b = orc.sample_lists(2, 1, np.arange(m, dtype=np.int32), P, T)
    share = np.array([len(np.intersect1d(a[i], b[i])) > 0 for i in range(m)])
    expect = 1 - math.comb(P - T, T) / math.comb(P, T)
    sd = math.sqrt(expect * (1 - expect) / m)
    assert abs(share.mean() - expect) < 5 * sd


def test_expected_bucket_pairs(orc):
    # E[sum_c C(|B_c|,2)] = C(m,2) T^2 / P
    P, T, m = 400, 9, 3000
    tot = []
    for seed in range(6):
        lists = orc.sample_lists(seed, 1, np.arange(m, dtype=np.int32), P, T)
        cnt = np.bincount(lists.ravel(), minlength=P).astype(np.int64)
        tot.append(int((cnt * (cnt - 1) // 2).sum()))
    expect = math.comb(m, 2) * T * T / P
    assert abs(np.mean(tot) / expect - 1) < 0.01


def test_lists_depend_on_original_id_only(orc):
    ids = np.array([5, 17, 3, 99, 42], dtype=np.int32)
    perm = np.array([3, 0, 4, 1, 2])
    a = orc.sample_lists(77, 2, ids, 100, 8)
    b = orc.sample_lists(77, 2, ids[perm], 100, 8)
    assert np.array_equal(a[perm], b)


def test_keys_separate_streams(orc):
    base = orc.sample_list(1, 1, 1, 10_000, 20)
    assert not np.array_equal(base, orc.sample_list(2, 1, 1, 10_000, 20))  # seed
    assert not np.array_equal(base, orc.sample_list(1, 2, 1, 10_000, 20))  # iteration
    assert not np.array_equal(base, orc.sample_list(1, 1, 2, 10_000, 20))  # vertex
    assert orc.priority(1, 1, 1) != orc.hash64(1, 1, 0, 1, 0x4C495354)  # tags differ


def test_philox_bit_balance_and_avalanche(orc):
    rng = np.random.default_rng(0)
    words = []
    flips = []
    for _ in range(400):
        ctr = rng.integers(0, 2**32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2**32, 2, dtype=np.uint64).astype(np.uint32)
        out = orc.philox4x32_10(ctr, key)
        words.append(out)
        c2 = ctr.copy()
        bit = rng.integers(128)
        c2[bit // 32] ^= np.uint32(1 << (bit % 32))
        out2 = orc.philox4x32_10(c2, key)
        flips.append(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(out, out2)))
    bits = np.unpackbits(np.array(words, dtype=">u4").view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.01
    assert abs(np.mean(flips) - 64) < 2.0  # half of 128 output bits flip


def test_priorities_uniform_order(orc):
    # the random static order: each of 3! orders of 3 vertices equally likely
    counts = {}
    for seed in range(6000):
        p = [orc.priority(seed, 1, v) for v in range(3)]
        key = tuple(np.argsort(p))
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 6
    chi2, pv = stats.chisquare(list(counts.values()))
    assert pv > 1e-4


def test_philox_known_answer_vectors(orc):
    """Philox4x32-10 against the known-answer vectors published with the
    generator (Salmon et al., SC'11; Random123): counters and keys of all
    zeros, all ones, and digits of pi."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(t, 16) for t in r]
        out = orc.philox4x32_10(np.array(w[:4], dtype=np.uint32), np.array(w[4:6], dtype=np.uint32))
        assert [int(v) for v in out] == w[6:10]
