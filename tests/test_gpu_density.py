"""The other density functions (Sec. 4.2 normalized; appendix A exp-sum,
sum-exp, sum), the local center function and clustering from given centers,
against the oracle.  The GPU computes densities in float32 from its float32
kNN distances, the oracle in FP64: densities agree within float32 rounding and
the density order agrees wherever the oracle's own gap is above that rounding.
Logic on identical inputs (local centers from the same keys, labels from the
same centers) is bit-exact."""
import numpy as np
import pytest
import torch

import oracle
from oracle import metrics
from paper_2312_03940_amd import datagen, pecann

pytestmark = pytest.mark.gpu
FNS = ["kth", "normalized", "exp-sum", "sum-exp", "sum"]


@pytest.fixture(scope="module")
def case():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    dev = torch.device("cuda:0")
    X, _ = datagen.mixture(3000, 16, 8, seed=77, grid=511)
    X = X / 64.0  # keep exp(-D^2) away from underflow; exact in binary
    k = 8
    ref_idx, ref_dist = oracle.knn(oracle.Points(X), k)
    ds = pecann.Dataset(torch.from_numpy(X).to(dev), "l2", "f32")
    idx, dist, rho, key = pecann.knn_density(ds, k)
    torch.cuda.synchronize()
    assert np.array_equal(idx.cpu().numpy(), ref_idx)  # exact kNN, integer grid
    return dict(X=X, k=k, ds=ds, idx=idx, dist=dist, rho=rho, key=key, ref_idx=ref_idx,
                ref_dist=ref_dist, dev=dev)


def _order_ok(ref_rho, gpu_key, rtol):
    """GPU order (by key) vs the oracle's density order; a swap is allowed only
    between points whose oracle densities are within rtol."""
    order_g = np.lexsort((np.arange(len(gpu_key)), gpu_key.astype(np.uint64)))
    order_o, _ = oracle.rank_from_rho(ref_rho)
    bad = np.nonzero(order_g != order_o)[0]
    a, b = ref_rho[order_g[bad]], ref_rho[order_o[bad]]
    return np.all(np.abs(a - b) <= rtol * np.maximum(np.abs(a), np.abs(b)))


@pytest.mark.parametrize("fn", FNS)
def test_density_function_matches_oracle(case, fn):
    ref = oracle.density(case["ref_idx"], case["ref_dist"], fn)
    out = (torch.empty_like(case["rho"]), case["key"].clone()) if fn == "kth" else None
    rho, key = pecann.density(case["idx"], case["dist"], fn, out=out)
    rho, key = rho.cpu().numpy(), key.cpu().numpy()
    assert np.allclose(rho, ref, rtol=2e-5, atol=0), fn
    assert _order_ok(ref, key, 4e-5), fn
    # keys: smaller key = higher density, ties to the lower index
    order = np.lexsort((np.arange(len(key)), key.astype(np.uint64)))
    assert np.all(np.diff(rho[order]) <= 0)
    assert np.all((key & 0xffffffff) == np.arange(len(key)))


def test_local_centers_and_given_center_labels(case):
    rho, key = pecann.density(case["idx"], case["dist"], "exp-sum")
    dep, delta, _ = pecann.dependent_search(case["ds"], key, case["idx"], case["dist"])
    isc = pecann.local_centers(case["idx"], key, rho)
    rho_n, key_n, dep_n, delta_n, isc_n = (t.cpu().numpy() for t in (rho, key, dep, delta, isc))
    rank_g = np.empty(len(key_n), np.int64)
    rank_g[np.lexsort((np.arange(len(key_n)), key_n.astype(np.uint64)))] = np.arange(len(key_n))
    # same keys -> same local centers as the oracle's definition
    assert np.array_equal(isc_n.astype(bool), oracle.local_centers(case["ref_idx"], rank_g, rho_n))
    assert isc_n[np.argmin(rank_g)]  # the densest point
    # same dependents and centers -> same labels
    labels, isc2 = pecann.cluster(rho, dep, delta, center_mode=pecann.CENTER_GIVEN,
                                  out=(torch.empty_like(dep), isc.clone()))
    ref_labels, ref_isc = oracle.cluster(rho_n, dep_n, delta_n, center_mode=oracle.CENTER_GIVEN,
                                         centers=isc_n)
    assert np.array_equal(labels.cpu().numpy(), ref_labels)
    assert np.array_equal(isc2.cpu().numpy().astype(bool), ref_isc)
    # noise points are never centers and label themselves
    rho_min = float(np.sort(rho_n)[50])
    labels3, isc3 = pecann.cluster(rho, dep, delta, center_mode=pecann.CENTER_GIVEN, rho_min=rho_min,
                                   out=(torch.empty_like(dep), isc.clone()))
    noise = rho_n < rho_min
    assert not isc3.cpu().numpy()[noise].any()
    assert np.array_equal(labels3.cpu().numpy()[noise], np.nonzero(noise)[0])


@pytest.mark.parametrize("fn", ["normalized", "exp-sum"])
def test_dpc_with_other_density_matches_oracle(case, fn):
    # exact DPC with another density and product centers: labels against the
    # oracle's exact DPC with the same density (ARI; decisions near float32
    # ties may differ)
    rho, key = pecann.density(case["idx"], case["dist"], fn)
    dep, delta, _ = pecann.dependent_search(case["ds"], key, case["idx"], case["dist"])
    labels, _ = pecann.cluster(rho, dep, delta, n_c=8)
    ref_rho = oracle.density(case["ref_idx"], case["ref_dist"], fn)
    _, rank = oracle.rank_from_rho(ref_rho)
    rdep, rdelta = oracle.dependent_exact(oracle.Points(case["X"]), rank)
    rlab, _ = oracle.cluster(ref_rho, rdep, rdelta, n_c=8)
    assert metrics.ari(labels.cpu().numpy(), rlab) >= 0.99
    agree = np.mean(dep.cpu().numpy() == rdep)
    assert agree >= 0.99, agree


def test_kth_density_keeps_the_knn_keys(case):
    # the kth function's order is the k-th neighbour's measure with ties to the
    # lower index (Sec. 3 ranking); its keys stay those of the kNN search, so
    # both entry points hand the dependent search the same order.  On this
    # integer grid every D_k^2 is an exact integer: the order equals the
    # oracle's (D_k, index) rank exactly, near-ties of 1 / D_k included.
    rho, key = pecann.density(case["idx"], case["dist"], "kth",
                              out=(torch.empty_like(case["rho"]), case["key"].clone()))
    assert torch.equal(key, case["key"])
    assert torch.equal(rho, case["rho"])
    key_n = key.cpu().numpy()
    order_g = np.lexsort((np.arange(len(key_n)), key_n.astype(np.uint64)))
    order_o, _ = oracle.rank_from_dk(case["ref_dist"][:, case["k"] - 1])
    assert np.array_equal(order_o, order_g)
    with pytest.raises(ValueError):
        pecann.density(case["idx"], case["dist"], "kth")
