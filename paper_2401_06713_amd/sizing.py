"""Size of the conflict graph before it is built (Sec. IV-A and its analysis;
the memory bound of Alg. 3).

A pair joined by the relation conflicts when the two colour lists share a
colour.  Lists are uniform T-subsets of a palette of P colours (Floyd
sampling), so two lists are disjoint with probability C(P-T, T) / C(P, T)
and

    E|E_c| = C(m, 2) * rho * (1 - C(P-T, T) / C(P, T)),

with rho the fraction of vertex pairs the relation joins.  rho is what the
feature kernel already estimates from 4096 keyed random pairs
(`Picasso.features(...)[3]`), so the CSR can be sized, and a palette chosen
under a memory budget, before the count pass runs.  Host arithmetic only.
"""
from __future__ import annotations

import math


def pair_share(P: int, T: int) -> float:
    """Probability that two independent uniform T-subsets of P colours meet."""
    if T <= 0 or P <= 0:
        return 0.0
    if 2 * T > P:
        return 1.0
    # C(P-T, T) / C(P, T) = ((P-T)!)^2 / ((P-2T)! P!)
    log_disjoint = 2 * math.lgamma(P - T + 1) - math.lgamma(P - 2 * T + 1) - math.lgamma(P + 1)
    return 1.0 - math.exp(log_disjoint)


def expected_conflict_edges(m: int, P: int, T: int, density: float) -> float:
    """Expected undirected conflict edges of an iteration with m vertices."""
    return m * (m - 1) / 2.0 * density * pair_share(P, T)


def csr_bytes(m: int, edges: float) -> float:
    """Device bytes of the CSR the library writes: int64 row pointers and two
    int32 column indices per undirected edge."""
    return 8.0 * (m + 1) + 8.0 * edges
