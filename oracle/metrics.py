"""Evaluation metrics of the oracle (TEST INFRASTRUCTURE ONLY; see oracle/__init__.py).

* ``ari``          -- adjusted Rand index in the Hubert-Arabie form the paper uses to
                      compare a clustering with the exact one (Sec. 6.1, Evaluation).
* ``recall_at_k``  -- tie-tolerant recall of approximate kNN lists: a returned point
                      counts when its exact distance is no larger than the exact k-th
                      neighbour distance (so ties at the k-th distance never cost recall).
* ``dependent_agreement`` -- fraction of points whose dependent point equals the exact one.
"""
from __future__ import annotations

import numpy as np

from . import Points, distance


def _pairs(x):
    x = np.asarray(x, dtype=np.int64)
    return x * (x - 1) // 2


def contingency(a, b):
    """Contingency counts n_ij of two labelings (int64)."""
    a = np.asarray(a)
    b = np.asarray(b)
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    m = np.zeros((ai.max() + 1, bi.max() + 1), dtype=np.int64)
    np.add.at(m, (ai, bi), 1)
    return m


def ari(a, b) -> float:
    """(sum C(n_ij,2) - E) / ((A+B)/2 - E), A = sum C(n_i*,2), B = sum C(n_*j,2),
    E = A*B / C(n,2).  A zero denominator only happens when both labelings are
    the same trivial partition (one cluster, or all singletons); it returns 1.0."""
    n = len(a)
    if n != len(b):
        raise ValueError("labelings differ in length")
    if n < 2:
        return 1.0
    m = contingency(a, b)
    s_ij = float(_pairs(m).sum())
    A = float(_pairs(m.sum(axis=1)).sum())
    B = float(_pairs(m.sum(axis=0)).sum())
    N2 = float(n) * (n - 1) / 2.0
    expected = A * B / N2
    mx = 0.5 * (A + B)
    if mx == expected:
        return 1.0
    return (s_ij - expected) / (mx - expected)


def recall_at_k(P: Points, queries, returned_ids, exact_dist, k: int) -> float:
    """Mean over queries of |{returned j != q, unique : D(q,j) <= d_k(q)}| / k, capped at k."""
    queries = np.asarray(queries, dtype=np.int64)
    returned_ids = np.asarray(returned_ids)
    exact_dist = np.asarray(exact_dist, dtype=np.float64)
    tot = 0
    for t, q in enumerate(queries):
        thr = exact_dist[t, k - 1]
        seen = set()
        c = 0
        for j in returned_ids[t, :k]:
            j = int(j)
            if j < 0 or j == q or j in seen:
                continue
            seen.add(j)
            if distance(P, int(q), j) <= thr:
                c += 1
        tot += min(c, k)
    return tot / (k * len(queries))


def dependent_agreement(dep_a, dep_b) -> float:
    dep_a = np.asarray(dep_a)
    dep_b = np.asarray(dep_b)
    return float(np.mean(dep_a == dep_b))
