"""The reverse prune's shortcut, checked as a model on the CPU.

When a target's list starts with the entries its previous RobustPrune
selected, the device prune forms only the distances between the other
candidates U (entries appended since, new sources) and all candidates, and
settles the greedy pass with a walk over U in (distance, index) order: a member
of U is dropped by a selected U member before it, or by a selected settled entry
before it; a settled entry is selected unless a selected U member before it
drops it.  The claim is that this equals the full greedy pass (DiskANN's
RobustPrune, Sec. 3.2) whenever the settled entries came from a prune with an
alpha no larger than the current one.  This test restates the walk in plain
Python and compares it with the oracle's RobustPrune on random float data,
with the alpha schedule of the two-pass build (1 then 1.2) and with equal
alphas; it also shows that the premise matters (calling appended entries
settled changes some results)."""
import numpy as np
import pytest

import oracle


def _walk(P, p, settled, others, alpha, R):
    d = {c: oracle.distance(P, p, c) for c in list(settled) + list(others)}
    order = sorted(d, key=lambda c: (d[c], c))
    pos = {c: i for i, c in enumerate(order)}
    sset = set(settled)
    upos = [c for c in order if c not in sset]
    uidx = {c: i for i, c in enumerate(upos)}
    kU = {c: set() for c in order}   # U members before c that would drop c
    cU = {c: set() for c in order}   # U members after c that c would drop
    for u in upos:
        for c in order:
            if c == u:
                continue
            m = oracle.distance(P, u, c)
            if pos[u] < pos[c]:
                if alpha * m <= d[c]:
                    kU[c].add(uidx[u])
            elif alpha * m <= d[u]:
                cU[c].add(uidx[u])
    sel = set()
    for t, u in enumerate(upos):
        dead = bool(kU[u] & sel)
        for c in order:
            if dead or pos[c] >= pos[u]:
                break
            dead = c in sset and not (kU[c] & sel) and t in cU[c]
        if not dead:
            sel.add(t)
    out = [c for c in order if ((uidx[c] in sel) if c not in sset else not (kU[c] & sel))]
    return out[:R]


def _cases(seed, trials, alphas, R):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(400, 8)).astype(np.float32)
    X[200:] += 3.0  # two blobs: some candidates far, some near
    P = oracle.Points(X)
    for _ in range(trials):
        p = int(rng.integers(len(X)))
        pool = rng.permutation(np.setdiff1d(np.arange(len(X)), [p]))
        first = pool[:int(rng.integers(R, 3 * R))]
        settled = [int(c) for c in oracle.robust_prune(P, p, first, alphas[0], R)]
        rest = [int(c) for c in pool if int(c) not in set(settled)]
        n_app = int(rng.integers(0, R - len(settled) + 1))
        n_new = int(rng.integers(1, 40))
        yield P, p, settled, rest[:n_app], rest[n_app:n_app + n_new]


@pytest.mark.parametrize("alphas", [(1.0, 1.2), (1.2, 1.2), (1.0, 1.0)])
def test_walk_equals_full_greedy(alphas):
    R = 24
    for P, p, settled, appended, new in _cases(7, 60, alphas, R):
        cand = settled + appended + new
        full = [int(c) for c in oracle.robust_prune(P, p, np.array(cand), alphas[1], R)]
        assert _walk(P, p, settled, appended + new, alphas[1], R) == full


def test_walk_needs_settled_entries():
    # appended entries were never checked against each other: calling them
    # settled must change some results, or the test above would prove nothing
    R = 24
    differ = 0
    for P, p, settled, appended, new in _cases(11, 60, (1.0, 1.2), R):
        if not appended:
            continue
        cand = settled + appended + new
        full = [int(c) for c in oracle.robust_prune(P, p, np.array(cand), 1.2, R)]
        differ += _walk(P, p, settled + appended, new, 1.2, R) != full
    assert differ > 0
