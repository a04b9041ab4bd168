"""Dendrogram re-cut (Sec. 1; Sec. 6 varying n_c): densities and dependent points
are computed once; each cut is one pecann_cluster call.  Product-center cuts are
nested (the n_c largest gamma include the n_c - 1 largest), so every cluster of a
finer cut lies inside one cluster of a coarser cut; each cut equals the oracle's
exact DPC with that n_c (integer grid: bit-exact)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2312_03940_amd import datagen, pecann

pytestmark = pytest.mark.gpu


def test_recut_sweep_nested_and_exact():
    dev = torch.device("cuda:0")
    X, _ = datagen.config1(integer_grid=True)
    k = 10
    ds = pecann.Dataset(torch.from_numpy(X).to(dev), "l2", "f32")
    idx, dist, rho, key = pecann.knn_density(ds, k)
    dep, delta, _ = pecann.dependent_search(ds, key, idx, dist)
    ref = oracle.exact_dpc(X, k=k, n_c=1)
    prev = None
    for n_c in [1, 2, 3, 5, 8, 10, 13, 20, 40]:
        labels, isc = pecann.cluster(rho, dep, delta, n_c=n_c)
        lab = labels.cpu().numpy()
        assert len(np.unique(lab)) == n_c and int(isc.sum()) == n_c
        rlab, _ = oracle.cluster(ref["rho"], ref["dep"], ref["delta"], n_c=n_c)
        assert np.array_equal(lab, rlab), n_c
        if prev is not None:  # nested: each finer cluster maps to one coarser cluster
            pairs = np.unique(np.stack([lab, prev]), axis=1)
            assert len(np.unique(pairs[0])) == pairs.shape[1]
        prev = lab
