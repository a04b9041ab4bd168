"""Plain FP64 CPU oracle for the PECANN density-peaks hot path (arXiv 2312.03940).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_2312_03940_amd``) never imports it, and the two share no code: the only
module both sides use is the seeded input generator, which holds none of the
method's arithmetic.

The heavy loops live in ``dpc_oracle.c`` (plain C, FP64, direct differences,
OpenMP across independent queries only).  This module marshals numpy arrays into
it and composes the steps of Alg. 2 in the paper's order:

* ``exact_dpc``     -- the paper's BruteForce instantiation ("exact DPC", Sec. 6.1):
                       exact kNN, kth density, exact dependent points (Def. 1),
                       noise / centers / labels (Alg. 2);
* ``anns_dpc``      -- the same steps over a graph index: greedy beam search
                       (Alg. 1) for the kNN, ComputeDepPts (Alg. 3) for the
                       dependent points;
* ``vamana_build``  -- batched Vamana insertion with RobustPrune (Sec. 3.2);
* ``ari`` / ``recall_at_k`` -- the evaluation metrics (Sec. 6.1).

No function here has a GPU counterpart in its call graph.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

__all__ = [
    "build_oracle", "load", "Points", "knn", "rank_from_dk", "dependent_exact",
    "cluster", "greedy_search", "robust_prune", "vamana_build", "dependent_alg3",
    "exact_dpc", "anns_dpc", "distance", "num_threads", "batch_schedule",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpc_oracle.c")
# PECANN_ORACLE_LIB: another build of dpc_oracle.c (the sanitizer test's)
_LIB = os.environ.get("PECANN_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

L2, COSINE = 0, 1
F32, U8 = 0, 1


def build_oracle(force: bool = True) -> str:
    """Compile dpc_oracle.c into liboracle.so (portable x86-64-v3 code)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _OPoints(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("stride", ctypes.c_int64)]


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_OPoints)
        vp = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_distance.argtypes = [P, i64, i64]
        lib.oracle_distance.restype = f64
        lib.oracle_knn.argtypes = [P, vp, i64, i32, vp, vp]
        lib.oracle_knn.restype = ctypes.c_int
        lib.oracle_rank.argtypes = [i64, vp, vp, vp]
        lib.oracle_rank.restype = None
        lib.oracle_dependent_exact.argtypes = [P, vp, vp, i64, vp, vp]
        lib.oracle_dependent_exact.restype = None
        lib.oracle_cluster.argtypes = [i64, vp, vp, vp, i32, i64, f64, f64, vp, vp]
        lib.oracle_cluster.restype = ctypes.c_int
        lib.oracle_greedy_search.argtypes = [P, vp, vp, i32, i64, i64, vp, i32, i32, i32,
                                             vp, vp, vp, vp, i32, vp]
        lib.oracle_greedy_search.restype = i32
        lib.oracle_robust_prune.argtypes = [P, i64, vp, i32, f64, i32, vp]
        lib.oracle_robust_prune.restype = i32
        lib.oracle_vamana_build.argtypes = [P, i32, i32, f64, vp, i32, i64, i32, i32, vp, i64,
                                            vp, vp, vp]
        lib.oracle_vamana_build.restype = ctypes.c_int
        lib.oracle_dependent_alg3.argtypes = [P, vp, vp, i32, vp, vp, i32, i32, i64, i32,
                                              i32, vp, vp, vp, i32]
        lib.oracle_dependent_alg3.restype = i32
        lib.oracle_nndescent.argtypes = [P, i32, i32, f64, i32, f64, i32, vp, vp, vp, vp, vp, vp]
        lib.oracle_nndescent.restype = ctypes.c_int
        lib.oracle_density.argtypes = [i64, i32, i32, vp, vp, vp]
        lib.oracle_density.restype = ctypes.c_int
        lib.oracle_rank_density.argtypes = [i64, vp, vp, vp]
        lib.oracle_rank_density.restype = None
        lib.oracle_local_centers.argtypes = [i64, i32, vp, vp, vp, f64, vp]
        lib.oracle_local_centers.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Points:
    """A point set as the oracle sees it: float32 or uint8 rows, L2 or cosine."""

    def __init__(self, X: np.ndarray, metric: int = L2):
        if X.dtype == np.uint8:
            dt = U8
        elif X.dtype == np.float32:
            dt = F32
        else:
            raise TypeError("oracle points must be float32 or uint8")
        self.X = np.ascontiguousarray(X)
        self.n, self.d = self.X.shape
        self.metric = metric
        self.s = _OPoints(self.X.ctypes.data, self.n, self.d, dt, metric, self.d)

    @property
    def ref(self):
        return ctypes.byref(self.s)


def num_threads() -> int:
    return int(load().oracle_num_threads())


def distance(P: Points, i: int, j: int) -> float:
    return float(load().oracle_distance(P.ref, i, j))


def knn(P: Points, k: int, queries=None):
    """Exact kNN, self excluded, (distance, index) ascending.  -> (idx int64, dist f64)."""
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = P.n if q is None else len(q)
    idx = np.empty((nq, k), dtype=np.int64)
    dist = np.empty((nq, k), dtype=np.float64)
    if load().oracle_knn(P.ref, _ptr(q), nq, k, _ptr(idx), _ptr(dist)) != 0:
        raise ValueError("oracle_knn: k out of range")
    return idx, dist


def rank_from_dk(dk: np.ndarray):
    """Total density order: (D_k, index) ascending.  -> (order, rank)."""
    dk = np.ascontiguousarray(dk, dtype=np.float64)
    n = len(dk)
    order = np.empty(n, dtype=np.int64)
    rank = np.empty(n, dtype=np.int64)
    load().oracle_rank(n, _ptr(dk), _ptr(order), _ptr(rank))
    return order, rank


def dependent_exact(P: Points, rank: np.ndarray, queries=None):
    """Def. 1 by brute force.  -> (dep int64 (-1 = none), delta f64 (+inf = none))."""
    rank = np.ascontiguousarray(rank, dtype=np.int64)
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = P.n if q is None else len(q)
    dep = np.empty(nq, dtype=np.int64)
    delta = np.empty(nq, dtype=np.float64)
    load().oracle_dependent_exact(P.ref, _ptr(rank), _ptr(q), nq, _ptr(dep), _ptr(delta))
    return dep, delta


DENSITY_FNS = {"kth": 0, "normalized": 1, "exp-sum": 2, "sum-exp": 3, "sum": 4}
CENTER_PRODUCT, CENTER_THRESHOLD, CENTER_GIVEN = 0, 1, 2


def density(knn_idx, knn_dist, fn="kth"):
    """Density of every point from its k nearest neighbours (Sec. 4.2; App. A).
    -> rho float64 [n]."""
    idx = np.ascontiguousarray(knn_idx, dtype=np.int64)
    dist = np.ascontiguousarray(knn_dist, dtype=np.float64)
    n, k = idx.shape
    rho = np.empty(n, dtype=np.float64)
    if load().oracle_density(n, k, DENSITY_FNS[fn], _ptr(idx), _ptr(dist), _ptr(rho)) != 0:
        raise ValueError(fn)
    return rho


def rank_from_rho(rho):
    """Density order of any density function: rho descending, ties to the lower index.
    -> (order, rank)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    n = len(rho)
    order = np.empty(n, dtype=np.int64)
    rank = np.empty(n, dtype=np.int64)
    load().oracle_rank_density(n, _ptr(rho), _ptr(order), _ptr(rank))
    return order, rank


def local_centers(knn_idx, rank, rho, rho_min=0.0):
    """Non-noise points ranked above all their k nearest neighbours (App. A). -> bool [n]."""
    idx = np.ascontiguousarray(knn_idx, dtype=np.int64)
    rank = np.ascontiguousarray(rank, dtype=np.int64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    n, k = idx.shape
    isc = np.zeros(n, dtype=np.uint8)
    load().oracle_local_centers(n, k, _ptr(idx), _ptr(rank), _ptr(rho), ctypes.c_double(rho_min),
                                _ptr(isc))
    return isc.astype(bool)


def cluster(rho, dep, delta, n_c=1, center_mode=0, delta_min=0.0, rho_min=0.0, centers=None):
    """Noise, centers and root labels (Alg. 2).  center_mode 2 takes the given centers.
    -> (labels int64, is_center bool)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    dep = np.ascontiguousarray(dep, dtype=np.int64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    n = len(rho)
    labels = np.empty(n, dtype=np.int64)
    isc = np.zeros(n, dtype=np.uint8) if centers is None else \
        np.ascontiguousarray(centers, dtype=np.uint8).copy()
    rc = load().oracle_cluster(n, _ptr(rho), _ptr(dep), _ptr(delta), center_mode, n_c,
                               delta_min, rho_min, _ptr(labels), _ptr(isc))
    if rc != 0:
        raise ValueError("oracle_cluster failed (cycle in dependent pointers?)")
    return labels, isc.astype(bool)


def greedy_search(P: Points, adj, deg, q: int, starts, L: int, k: int, excl: int = -1,
                  want_visited: bool = False):
    """Alg. 1.  -> (ids, dists) of the k closest, plus (visited ids, dists) if asked."""
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    deg = np.ascontiguousarray(deg, dtype=np.int32)
    R = adj.shape[1]
    st = np.ascontiguousarray(starts, dtype=np.int64)
    ids = np.empty(max(k, 1), dtype=np.int64)
    ds = np.empty(max(k, 1), dtype=np.float64)
    nvis = ctypes.c_int32(0)
    vis_ids = np.empty(P.n, dtype=np.int64)
    vis_d = np.empty(P.n, dtype=np.float64)
    c = load().oracle_greedy_search(P.ref, _ptr(adj), _ptr(deg), R, q, excl, _ptr(st), len(st),
                                    L, k, _ptr(ids), _ptr(ds), _ptr(vis_ids), _ptr(vis_d),
                                    P.n, ctypes.byref(nvis))
    if c < 0:
        raise MemoryError("oracle_greedy_search")
    out = (ids[:c].copy(), ds[:c].copy())
    if want_visited:
        nv = nvis.value
        return out + (vis_ids[:nv].copy(), vis_d[:nv].copy())
    return out


def robust_prune(P: Points, p: int, cand, alpha: float, R: int):
    cand = np.ascontiguousarray(cand, dtype=np.int64)
    out = np.empty(max(R, 1), dtype=np.int64)
    c = load().oracle_robust_prune(P.ref, p, _ptr(cand), len(cand), alpha, R, _ptr(out))
    if c < 0:
        raise MemoryError("oracle_robust_prune")
    return out[:c].copy()


def batch_schedule(n: int, max_batch: int = 0):
    """Batch boundaries of the first insertion pass: perm[0] alone, then 1, 2, 4, ... capped
    at max_batch (0: floor(n / 50), the paper's 0.02 n)."""
    cap = max(1, max_batch if max_batch > 0 else n // 50)
    bounds = [(0, 1)]
    ins, b = 1, 1
    while ins < n:
        nb = min(b, cap, n - ins)
        bounds.append((ins, ins + nb))
        ins += nb
        b *= 2
    return bounds


def vamana_build(P: Points, R: int, L: int, alpha: float, perm, num_starts: int = 8,
                 max_batch: int = 0, passes: int = 2, max_vis: int = 0, want_batches: bool = False):
    """passes=2: DiskANN's schedule (alpha = 1, then alpha); passes=1: alpha only.
    max_vis > 0 keeps the max_vis closest points of each visited set (0: all).
    want_batches: also return the batches the build ran, as (pass, first, size) rows."""
    perm = np.ascontiguousarray(perm, dtype=np.int64)
    adj = np.empty((P.n, R), dtype=np.int32)
    deg = np.empty(P.n, dtype=np.int32)
    cap = 4 * P.n + 64
    log = np.empty((cap, 3), dtype=np.int64)
    nlog = ctypes.c_int64(0)
    if load().oracle_vamana_build(P.ref, R, L, alpha, _ptr(perm), num_starts, max_batch,
                                  passes, max_vis, _ptr(log), cap, ctypes.byref(nlog),
                                  _ptr(adj), _ptr(deg)) != 0:
        raise MemoryError("oracle_vamana_build")
    if want_batches:
        return adj, deg, log[:min(nlog.value, cap)].copy()
    return adj, deg


def nndescent(P: Points, init, K: int, R: int, alpha: float, max_iters: int, delta: float = 0.0):
    """NN-descent lists in synchronous rounds, then RobustPrune(list u reverse list).
    init: [num_repeats, n, K] (or [n, K]) distinct ids other than the row's own.
    -> (adj int32 [n, R], deg int32 [n], list_idx int64 [n, K], list_dist float64 [n, K],
        rounds int32 [num_repeats])."""
    init = np.ascontiguousarray(init, dtype=np.int64)
    if init.ndim == 2:
        init = init[None]
    reps = init.shape[0]
    assert init.shape[1:] == (P.n, K)
    adj = np.empty((P.n, R), dtype=np.int32)
    deg = np.empty(P.n, dtype=np.int32)
    li = np.empty((P.n, K), dtype=np.int64)
    ld = np.empty((P.n, K), dtype=np.float64)
    rounds = np.zeros(reps, dtype=np.int32)
    if load().oracle_nndescent(P.ref, K, R, alpha, max_iters, delta, reps, _ptr(init), _ptr(adj),
                               _ptr(deg), _ptr(li), _ptr(ld), _ptr(rounds)) != 0:
        raise ValueError("oracle_nndescent: bad init or allocation failure")
    return adj, deg, li, ld, rounds


def dependent_alg3(P: Points, adj, deg, rank, knn_idx, L_d: int, threshold: int,
                   L_min: int = 0, kdep_cap: int = 1 << 30):
    """Alg. 3 (adj=None: the brute-force instantiation).  -> (dep, delta, rounds, |U| per round)."""
    rank = np.ascontiguousarray(rank, dtype=np.int64)
    knn_idx = np.ascontiguousarray(knn_idx, dtype=np.int64)
    k = knn_idx.shape[1]
    n = P.n
    dep = np.empty(n, dtype=np.int64)
    delta = np.empty(n, dtype=np.float64)
    rounds_out = np.zeros(64, dtype=np.int64)
    if adj is not None:
        adj = np.ascontiguousarray(adj, dtype=np.int32)
        deg = np.ascontiguousarray(deg, dtype=np.int32)
        R = adj.shape[1]
    else:
        R = 0
    r = load().oracle_dependent_alg3(P.ref, _ptr(adj), _ptr(deg), R, _ptr(rank), _ptr(knn_idx),
                                     k, L_d, threshold, L_min, kdep_cap, _ptr(dep), _ptr(delta),
                                     _ptr(rounds_out), 64)
    if r < 0:
        raise MemoryError("oracle_dependent_alg3")
    return dep, delta, r, rounds_out[: r + 1].copy()


def exact_dpc(X: np.ndarray, k: int, n_c: int, metric: int = L2, center_mode: int = 0,
              delta_min: float = 0.0, rho_min: float = 0.0):
    """The paper's exact DPC (BruteForce instantiation of Alg. 2) with the kth density."""
    P = Points(X, metric)
    idx, dist = knn(P, k)
    dk = dist[:, k - 1]
    with np.errstate(divide="ignore"):
        rho = 1.0 / dk
    order, rank = rank_from_dk(dk)
    dep, delta = dependent_exact(P, rank)
    labels, isc = cluster(rho, dep, delta, n_c, center_mode, delta_min, rho_min)
    return dict(knn_idx=idx, knn_dist=dist, dk=dk, rho=rho, order=order, rank=rank, dep=dep,
                delta=delta, labels=labels, is_center=isc)


def anns_dpc(X: np.ndarray, k: int, n_c: int, R: int, L_build: int, alpha: float, perm,
             L_search: int, L_d: int, threshold: int, num_starts: int = 8,
             max_batch: int = 0, kdep_cap: int = 1 << 30, metric: int = L2,
             center_mode: int = 0, delta_min: float = 0.0, rho_min: float = 0.0,
             passes: int = 2):
    """Alg. 2 over a Vamana index: build, Alg. 1 kNN from S = {i}, kth density, Alg. 3, cluster."""
    P = Points(X, metric)
    adj, deg = vamana_build(P, R, L_build, alpha, perm, num_starts, max_batch, passes)
    n = P.n
    idx = np.empty((n, k), dtype=np.int64)
    dist = np.empty((n, k), dtype=np.float64)
    for i in range(n):
        ids, ds = greedy_search(P, adj, deg, i, [i], max(L_search, k), k, excl=i)
        if len(ids) < k:  # too few results: exact search for this query (Sec. 4.1)
            ids2, ds2 = knn(P, k, [i])
            ids, ds = ids2[0], ds2[0]
        idx[i], dist[i] = ids, ds
    dk = dist[:, k - 1]
    with np.errstate(divide="ignore"):
        rho = 1.0 / dk
    order, rank = rank_from_dk(dk)
    dep, delta, rounds, ucount = dependent_alg3(P, adj, deg, rank, idx, L_d, threshold,
                                                L_search, kdep_cap)
    labels, isc = cluster(rho, dep, delta, n_c, center_mode, delta_min, rho_min)
    return dict(adj=adj, deg=deg, knn_idx=idx, knn_dist=dist, dk=dk, rho=rho, rank=rank,
                dep=dep, delta=delta, rounds=rounds, ucount=ucount, labels=labels,
                is_center=isc)
