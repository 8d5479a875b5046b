"""The conflict-graph size predicted before the count pass against the
oracle's exact edge counts (host arithmetic; no GPU)."""
import math

import numpy as np
import pytest

from paper_2401_06713_amd import sizing
from paper_2401_06713_amd import workloads as wl


def test_pair_share_small_cases_by_enumeration():
    import itertools
    for P, T in ((5, 2), (6, 3), (7, 2), (4, 3)):
        subsets = list(itertools.combinations(range(P), T))
        meet = sum(1 for a in subsets for b in subsets if set(a) & set(b))
        assert sizing.pair_share(P, T) == pytest.approx(meet / len(subsets) ** 2, rel=1e-12)
    assert sizing.pair_share(10, 10) == 1.0 and sizing.pair_share(10, 0) == 0.0


@pytest.mark.parametrize("n,q,probs,rel,frac,alpha", [
    (2000, 16, (0.25, 0.25, 0.25, 0.25), 0, 0.125, 2.0),
    (3000, 48, (0.7, 0.1, 0.1, 0.1), 0, 0.125, 2.0),
    (2500, 40, (0.85, 0.05, 0.05, 0.05), 1, 0.05, 3.0),
    (2000, 30, (0.6, 0.1, 0.2, 0.1), 2, 0.25, 1.0),
])
def test_predicted_edges_match_oracle(orc, n, q, probs, rel, frac, alpha):
    x, z = wl.pauli_strings(n, q, probs, seed=n + q)
    ids = np.arange(n, dtype=np.int32)
    P, T = orc.params(n, frac, alpha)
    rho = orc.features(x, z, q, ids, 3, 1, rel)[3]
    predicted = sizing.expected_conflict_edges(n, P, T, rho)
    lists = orc.sample_lists(3, 1, ids, P, T)
    _, actual, _ = orc.conflict_edges_bucketed(orc.decode(x, z, q), ids, lists, P, rel, want_edges=False)
    # rho is a sample mean over 4096 pairs: allow four standard errors, plus 2%
    se = math.sqrt(max(rho * (1 - rho), 1e-4) / 4096) / max(rho, 1e-3)
    assert abs(predicted / actual - 1) < 4 * se + 0.02, (predicted, actual, rho)
    assert sizing.csr_bytes(n, actual) == 8 * (n + 1) + 8 * actual


def test_pairs_sharing_a_vertex_are_independent():
    """Two lists drawn against a third: the events "meets u's list" are
    independent (every fixed T-subset is met with the same probability), so
    the conflict-edge count has variance C(m,2) rho s (1 - s) with no
    covariance terms; checked by enumeration of all triples of subsets."""
    import itertools
    for P, T in ((5, 2), (6, 2), (6, 3), (7, 3)):
        subsets = [set(c) for c in itertools.combinations(range(P), T)]
        n = len(subsets)
        s = sizing.pair_share(P, T)
        both = sum(1 for a in subsets for b in subsets for c in subsets if a & b and a & c)
        assert both / n**3 == pytest.approx(s * s, rel=1e-12)
