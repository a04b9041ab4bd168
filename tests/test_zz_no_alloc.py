"""pecann_cluster_noalloc (the entry point for callers that cannot allocate)
against pecann_cluster on the same inputs, through the C ABI: labels and
centers are integer work, so the bar is bit-exact.  Two calls in a row, the
second on a smaller input, show that the fixed scratch carries nothing from
one call to the next."""
import numpy as np
import pytest
import torch

from paper_2312_03940_amd import datagen, pecann

pytestmark = pytest.mark.gpu


def _forest(n, d, nc, seed, dev):
    X, _ = datagen.mixture(n, d, nc, seed=seed, grid=511)
    ds = pecann.Dataset(torch.from_numpy(X).to(dev), "l2", "f32")
    idx, dist, rho, key = pecann.knn_density(ds, 10)
    dep, delta, _ = pecann.dependent_search(ds, key, idx, dist)
    return rho, dep, delta


def _same(a, b):
    torch.cuda.synchronize()
    return torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_cluster_noalloc_matches_cluster_on_two_calls():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    dev = torch.device("cuda:0")
    big = _forest(20_000, 16, 12, 101, dev)
    small = _forest(3_001, 8, 5, 202, dev)
    for (rho, dep, delta), nc in ((big, 12), (small, 5)):
        ref = pecann.cluster(rho, dep, delta, n_c=nc)
        got = pecann.cluster_noalloc(rho, dep, delta, n_c=nc)
        assert _same(ref, got)
        assert int(got[1].sum()) == nc
    # the other center rule and a noise cutoff, again large then small
    for rho, dep, delta in (big, small):
        rmin = float(torch.quantile(rho.float(), 0.05))
        dmin = float(torch.quantile(delta[torch.isfinite(delta)].float(), 0.99))
        ref = pecann.cluster(rho, dep, delta, center_mode=pecann.CENTER_THRESHOLD, delta_min=dmin,
                             rho_min=rmin)
        got = pecann.cluster_noalloc(rho, dep, delta, center_mode=pecann.CENTER_THRESHOLD,
                                     delta_min=dmin, rho_min=rmin)
        assert _same(ref, got)


def test_cluster_noalloc_rejects_sizes_beyond_its_scratch():
    dev = torch.device("cuda:0")
    n = (1 << 21) + 1
    rho = torch.ones(n, dtype=torch.float32, device=dev)
    dep = torch.full((n,), -1, dtype=torch.int32, device=dev)
    with pytest.raises(pecann.PecannError, match="2097152"):
        pecann.cluster_noalloc(rho, dep, rho, n_c=1)
