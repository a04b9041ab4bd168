"""Pins of the oracle's batched Vamana build (Sec. 3.2 "Vamana Graph Construction",
the batching footnote of Sec. 4.1, DiskANN's RobustPrune that Sec. 3.2 adopts).

The oracle's build (`oracle_vamana_build`, plain C) is checked against things that
do not share its code:
  * a restatement written here in Python from the same passages, with sets and
    sorted lists instead of the C loops, on tiny integer-grid inputs where every
    distance is an exact square root of an integer (so both sides take the same
    decisions), over many insertion orders, batch caps, alpha and R;
  * a build derived by hand on five points of a line;
  * the batch schedule the C loop actually ran (its own log), against the
    paper's rule: the graph starts with the first point, then batches of
    doubling size from 1, capped; a second pass re-inserts every point in full
    batches;
  * the visited-set cap: when a search expands more points than the cap, the
    closest are kept.
"""
import math
from collections import defaultdict

import numpy as np
import pytest

import oracle
from paper_2312_03940_amd import datagen


def _dist(X, i, j):
    d = X[i].astype(np.float64) - X[j].astype(np.float64)
    return math.sqrt(float(np.dot(d, d)))


def _order(X, q):
    return lambda v: (_dist(X, q, v), v)


def _greedy_visited(X, graph, q, starts, L):
    """Alg. 1 as sets: the beam holds at most L points; each step expands the
    closest unexpanded beam point, unions its out-neighbours into the beam and
    keeps the L closest.  The query never enters its own beam; if it is a start
    it is expanded first.  Returns the expanded points other than q, in order."""
    key = _order(X, q)
    beam = {s for s in starts if s != q}
    beam = set(sorted(beam, key=key)[:L])
    expanded = set()
    order = []
    if q in starts:
        beam |= {v for v in graph[q] if v != q}
        beam = set(sorted(beam, key=key)[:L])
        expanded.add(q)
    while True:
        todo = [v for v in beam if v not in expanded]
        if not todo:
            return order
        p = min(todo, key=key)
        beam |= {v for v in graph[p] if v != q}
        expanded.add(p)
        order.append(p)
        beam = set(sorted(beam, key=key)[:L])


def _prune(X, p, cands, alpha, R):
    """DiskANN's RobustPrune: take the closest remaining candidate, drop every
    candidate c that it alpha-dominates (alpha * D(s, c) <= D(p, c)), repeat."""
    pool = sorted({c for c in cands if c != p and c >= 0}, key=_order(X, p))
    out = []
    while pool and len(out) < R:
        s = pool.pop(0)
        out.append(s)
        pool = [c for c in pool if not alpha * _dist(X, s, c) <= _dist(X, p, c)]
    return out


def _schedule(n, cap, passes):
    """(pass, first, size) of every batch: pass 0 starts the graph with perm[0]
    and inserts the rest in batches of 1, 2, 4, ... (at most cap); a later pass
    re-inserts all n points in batches of cap."""
    out = []
    for ps in range(passes):
        first, size = (1, 1) if ps == 0 else (0, cap)
        while first < n:
            b = min(size, cap, n - first)
            out.append((ps, first, b))
            first += b
            if ps == 0:
                size *= 2
    return out


def _restated_build(X, R, L, alpha, perm, num_starts, cap, passes, max_vis=0):
    n = len(X)
    graph = [[] for _ in range(n)]
    perm = [int(v) for v in perm]
    for ps, first, size in _schedule(n, cap, passes):
        a = 1.0 if (passes == 2 and ps == 0) else alpha
        in_graph = first if ps == 0 else n
        S = perm[:min(num_starts, in_graph)]
        snap = [list(row) for row in graph]  # every search of the batch sees this
        fresh = {}
        for p in perm[first:first + size]:
            V = _greedy_visited(X, snap, p, S, L)
            if max_vis and len(V) > max_vis:
                V = sorted(V, key=_order(X, p))[:max_vis]
            fresh[p] = _prune(X, p, V + snap[p], a, R)
        for p, out in fresh.items():
            graph[p] = out
        incoming = defaultdict(set)
        for p, out in fresh.items():
            for q in out:
                incoming[q].add(p)
        for q, srcs in incoming.items():
            add = [s for s in sorted(srcs) if s not in graph[q]]
            if len(graph[q]) + len(add) <= R:
                graph[q] = graph[q] + add
            else:
                graph[q] = _prune(X, q, graph[q] + add, a, R)
    return graph


def _as_lists(adj, deg):
    return [adj[i, :deg[i]].tolist() for i in range(len(deg))]


def test_restatement_matches_oracle_on_tiny_grids(oracle_lib):
    rng = np.random.default_rng(20231203)
    cases = 0
    for trial in range(150):
        n = int(rng.integers(3, 13))
        d = int(rng.integers(1, 4))
        X = rng.integers(0, 8, size=(n, d)).astype(np.float32)
        P = oracle.Points(X)
        perm = rng.permutation(n)
        R = int(rng.choice([2, 3]))
        L = int(rng.choice([2, 3, 5]))
        alpha = float(rng.choice([1.0, 1.2, 2.0]))
        cap = int(rng.choice([1, 2, 3]))
        ns = int(rng.choice([1, 2, 4]))
        passes = int(rng.choice([1, 2]))
        adj, deg = oracle.vamana_build(P, R, L, alpha, perm, num_starts=ns, max_batch=cap,
                                       passes=passes)
        want = _restated_build(X, R, L, alpha, perm, ns, cap, passes)
        assert _as_lists(adj, deg) == want, (trial, n, d, R, L, alpha, cap, ns, passes)
        assert np.all(adj[np.arange(R)[None, :] >= deg[:, None]] == -1)
        cases += 1
    assert cases == 150


def test_restatement_matches_oracle_larger(oracle_lib):
    # a few 40-point builds where batches hold many points (snapshot semantics matter)
    for seed in range(6):
        rng = np.random.default_rng(seed)
        X = rng.integers(0, 16, size=(40, 2)).astype(np.float32)
        P = oracle.Points(X)
        perm = rng.permutation(40)
        for alpha, cap in ((1.0, 8), (1.2, 5), (2.0, 16)):
            adj, deg = oracle.vamana_build(P, 4, 6, alpha, perm, num_starts=3, max_batch=cap,
                                           passes=2)
            assert _as_lists(adj, deg) == _restated_build(X, 4, 6, alpha, perm, 3, cap, 2)


def test_hand_derived_line_build(oracle_lib):
    # Points 0..4 at 0, 2, 3, 7, 8 on a line; one pass, alpha = 1, R = 2, L = 4,
    # the start set is {0}, batches [1], [2, 3], [4] (cap 2).
    #  [1]    search from 0 visits {0}; Nout(1) = {0}; reverse: Nout(0) = {1}.
    #  [2, 3] both search the graph 0 -> 1, 1 -> 0 and visit {0, 1}.
    #         p = 2: 1 is closest (D 1); D(1, 0) = 2 <= D(2, 0) = 3 drops 0.
    #         p = 3: 1 is closest (D 5); D(1, 0) = 2 <= 7 drops 0.
    #         reverse: 1 gets {2, 3}; {0, 2, 3} exceeds R, so prune 1 over it:
    #         2 (D 1) first, it drops 3 (D(2, 3) = 4 <= 5) but not 0 (3 > 2);
    #         then 0: Nout(1) = [2, 0].
    #  [4]    search from 0: expand 0 (adds 1), 1 (adds 2), 2; visits {0, 1, 2};
    #         2 (D 5) is closest and drops 1 (1 <= 6) and 0 (3 <= 8): Nout(4) = [2].
    #         reverse: Nout(2) = [1, 4] fits.
    # (Had p = 3 searched the live graph, where 1 already points to 2, it would
    # have visited 2 and linked to it instead.)
    X = np.array([[0.0], [2.0], [3.0], [7.0], [8.0]], dtype=np.float32)
    want = [[1], [2, 0], [1, 4], [1], [2]]
    P = oracle.Points(X)
    adj, deg = oracle.vamana_build(P, 2, 4, 1.0, np.arange(5), num_starts=1, max_batch=2,
                                   passes=1)
    assert _as_lists(adj, deg) == want
    assert _restated_build(X, 2, 4, 1.0, list(range(5)), 1, 2, 1) == want


def test_oracle_batch_log_is_the_paper_schedule(oracle_lib):
    for n, cap, passes in ((400, 3, 2), (70, 0, 2), (1000, 0, 1), (37, 5, 2), (2, 1, 2)):
        X = np.random.default_rng(n).integers(0, 9, size=(n, 2)).astype(np.float32)
        P = oracle.Points(X)
        _, _, log = oracle.vamana_build(P, 4, 8, 1.2, np.arange(n), num_starts=2,
                                        max_batch=cap, passes=passes, want_batches=True)
        eff = cap if cap > 0 else max(1, n // 50)  # the paper's 0.02 n by default
        assert [tuple(r) for r in log.tolist()] == _schedule(n, eff, passes)
    # the first pass doubles from 1 up to the cap (Sec. 4.1, footnote), the
    # second runs full batches
    X = np.random.default_rng(1).integers(0, 9, size=(3000, 2)).astype(np.float32)
    _, _, log = oracle.vamana_build(oracle.Points(X), 4, 8, 1.2, np.arange(3000), num_starts=2,
                                    max_batch=0, passes=2, want_batches=True)
    sizes0 = [int(s) for p, _, s in log if p == 0]
    sizes1 = [int(s) for p, _, s in log if p == 1]
    assert sizes0[:7] == [1, 2, 4, 8, 16, 32, 60] and set(sizes0[6:-1]) == {60}
    assert sum(sizes0) == 2999 and sum(sizes1) == 3000 and set(sizes1) == {60}


def test_visited_cap_keeps_the_closest(oracle_lib):
    rng = np.random.default_rng(7)
    hits = 0
    for trial in range(40):
        n = int(rng.integers(8, 25))
        X = rng.integers(0, 12, size=(n, 2)).astype(np.float32)
        P = oracle.Points(X)
        perm = rng.permutation(n)
        mv = int(rng.choice([1, 2, 3]))
        adj, deg = oracle.vamana_build(P, 3, 4, 1.2, perm, num_starts=2, max_batch=4,
                                       passes=2, max_vis=mv)
        want = _restated_build(X, 3, 4, 1.2, perm, 2, 4, 2, max_vis=mv)
        assert _as_lists(adj, deg) == want
        free = _restated_build(X, 3, 4, 1.2, perm, 2, 4, 2)
        hits += want != free
    assert hits > 0  # the cap changed some graphs, so the rule was exercised
