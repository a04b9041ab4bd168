"""Batches of independent instances (pecann_*_batched) against the oracle run
on each instance alone: every instance of a batch must give the same graph,
neighbours, dependent points and labels as the single-instance computation
(bit-exact on integer grids, where float32 and FP64 agree on every decision).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2312_03940_amd import datagen, pecann

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    pecann.load()
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _concat(sizes, ncs, d, seed):
    """Integer-grid mixtures of the given sizes, stacked; -> (X, offsets, parts)."""
    parts = [datagen.mixture(n, d, c, seed=seed + t, grid=511)[0] for t, (n, c) in
             enumerate(zip(sizes, ncs))]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return np.concatenate(parts), off, parts


def _shift(a, lo):
    """Local indices of one instance -> global (negative entries kept)."""
    a = np.asarray(a).astype(np.int64)
    return np.where(a >= 0, a + lo, a)


def test_batched_anns_matches_each_instance(dev):
    sizes, ks, ncs = [700, 1500, 2300], [5, 10, 8], [3, 6, 8]
    R, L, alpha, L_s, L_d, thr, cap, mb = 16, 32, 1.2, 24, 16, 20, 256, 200
    X, off, parts = _concat(sizes, ncs, 16, 40)
    perms = [datagen.permutation(n, 70 + t) for t, n in enumerate(sizes)]
    gperm = np.concatenate([p + off[t] for t, p in enumerate(perms)]).astype(np.int32)
    inst = pecann.Instances(off, k=ks, n_c=ncs)
    ds = pecann.Dataset(_t(X, dev), "l2", "f32")
    adj, deg = pecann.build_graph_batched(ds, inst, R, L, alpha, num_starts=4, perm=_t(gperm, dev),
                                          max_batch=mb)
    kmax = max(ks)
    idx, dist, rho, key = pecann.knn_density_batched(ds, inst, kmax, adj, deg, L_search=L_s)
    dep, delta, _ = pecann.dependent_search_batched(ds, inst, key, idx, dist, adj, deg, L_d=L_d,
                                                    L_search=L_s, threshold=thr, kdep_cap=cap)
    labels, isc = pecann.cluster_batched(inst, rho, dep, delta)
    adj, deg, idx, dist = _np(adj), _np(deg), _np(idx), _np(dist)
    dep, labels, isc = _np(dep), _np(labels), _np(isc)
    for t, n in enumerate(sizes):
        lo, hi, k = off[t], off[t + 1], ks[t]
        ref = oracle.anns_dpc(parts[t], k=k, n_c=ncs[t], R=R, L_build=L, alpha=alpha, perm=perms[t],
                              L_search=L_s, L_d=L_d, threshold=thr, num_starts=4, kdep_cap=cap,
                              max_batch=mb)
        assert np.array_equal(deg[lo:hi], ref["deg"]), t
        assert np.array_equal(adj[lo:hi], _shift(ref["adj"], lo)), t
        assert np.array_equal(idx[lo:hi, :k], _shift(ref["knn_idx"], lo)), t
        assert np.all(idx[lo:hi, k:] == -1) and np.all(np.isinf(dist[lo:hi, k:])), t
        assert np.allclose(dist[lo:hi, :k], ref["knn_dist"], rtol=1e-6), t
        assert np.array_equal(dep[lo:hi], _shift(ref["dep"], lo)), t
        assert np.array_equal(labels[lo:hi], _shift(ref["labels"], lo)), t
        assert np.array_equal(isc[lo:hi].astype(bool), ref["is_center"]), t


def test_batched_exact_matches_each_instance(dev):
    # the 4500-point instance takes the matrix-core scan, the others the direct kernel
    sizes, ks, ncs = [300, 4500, 1200], [7, 10, 4], [2, 5, 4]
    X, off, parts = _concat(sizes, ncs, 16, 90)
    inst = pecann.Instances(off, k=ks, n_c=ncs)
    ds = pecann.Dataset(_t(X, dev), "l2", "f32")
    kmax = max(ks)
    idx, dist, rho, key = pecann.knn_density_batched(ds, inst, kmax)
    dep, delta, _ = pecann.dependent_search_batched(ds, inst, key, idx, dist)
    labels, isc = pecann.cluster_batched(inst, rho, dep, delta)
    idx, dep, labels, key = _np(idx), _np(dep), _np(labels), _np(key)
    for t, n in enumerate(sizes):
        lo, hi, k = off[t], off[t + 1], ks[t]
        ref = oracle.exact_dpc(parts[t], k=k, n_c=ncs[t])
        assert np.array_equal(idx[lo:hi, :k], _shift(ref["knn_idx"], lo)), t
        order = np.lexsort((np.arange(n), key[lo:hi].astype(np.uint64) >> np.uint64(32)))
        assert np.array_equal(order, ref["order"]), t
        assert np.array_equal(dep[lo:hi], _shift(ref["dep"], lo)), t
        assert np.array_equal(labels[lo:hi], _shift(ref["labels"], lo)), t


def test_batched_seeded_order_matches_single_instance_seed(dev):
    # without perm, instance t shuffles with seed + t: instance 0 of a batch and a
    # single-instance build with the same seed insert in the same order
    sizes, ncs = [900, 600], [4, 3]
    X, off, parts = _concat(sizes, ncs, 8, 7)
    inst = pecann.Instances(off)
    ds = pecann.Dataset(_t(X, dev), "l2", "f32")
    adj_b, deg_b = pecann.build_graph_batched(ds, inst, 12, 24, 1.2, num_starts=4, seed=5,
                                              max_batch=100)
    ds0 = pecann.Dataset(_t(parts[0], dev), "l2", "f32")
    adj_0, deg_0 = pecann.build_graph(ds0, 12, 24, 1.2, num_starts=4, seed=5, max_batch=100)
    assert np.array_equal(_np(adj_b)[:900], _np(adj_0)) and np.array_equal(_np(deg_b)[:900], _np(deg_0))
    a1 = _np(adj_b)[900:]
    assert np.all((a1 == -1) | ((a1 >= 900) & (a1 < 1500)))  # edges stay inside the instance
