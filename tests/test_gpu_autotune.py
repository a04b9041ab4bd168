"""Launch tuning changes speed only: the graph, the kNN lists and the dependent
points are the same bytes under every setting; the autotuner picks, applies and
caches a setting."""
import json

import numpy as np
import pytest
import torch

from paper_2312_03940_amd import autotune, datagen, pecann

pytestmark = pytest.mark.gpu

# (hash bits build, hash bits search, grid per CU, prune tile steps)
SETTINGS = [(0, 0, 0, 0), (10, 13, 4, 4), (13, 10, 64, 2), (11, 12, 12, 4)]


def _step(ds, perm, k):
    adj, deg = pecann.build_graph(ds, 24, 48, 1.2, perm=perm)
    idx, dist, rho, key = pecann.knn_density(ds, k, adj, deg, L_search=48)
    dep, delta, _ = pecann.dependent_search(ds, key, idx, dist, adj, deg, L_d=32, L_search=48)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (adj, deg, idx, dist, key, dep, delta)]


@pytest.mark.parametrize("sdt", ["bf16", "u8", "f32"])
def test_tuning_does_not_change_results(sdt):
    dev = torch.device("cuda:0")
    X, _ = datagen.mixture(5000, 40, 10, seed=4, grid=255 if sdt == "u8" else None)
    x = torch.from_numpy(X.astype(np.uint8) if sdt == "u8" else X).to(dev)
    perm = torch.from_numpy(datagen.permutation(5000, 1)).to(dev)
    ds = pecann.Dataset(x, "l2", sdt)
    try:
        ref = None
        for hb, hs, g, ps in SETTINGS:
            pecann.set_tuning(hb, hs, g, 0, ps)
            assert pecann.get_tuning() == {"hash_bits_build": hb, "hash_bits_search": hs, "grid_per_cu": g,
                                           "scorer": 0, "prune_steps": ps}
            got = _step(ds, perm, 8)
            if ref is None:
                ref = got
            else:
                for a, b in zip(got, ref):
                    assert np.array_equal(a, b), (hb, hs, g, ps)
    finally:
        pecann.reset_tuning()


def test_autotune_picks_applies_and_caches(tmp_path):
    dev = torch.device("cuda:0")
    X, _ = datagen.mixture(4000, 32, 8, seed=6)
    ds = pecann.Dataset(torch.from_numpy(X).to(dev), "l2", "bf16")
    path = str(tmp_path / "tune.json")
    try:
        e = autotune.tune(ds, 24, 48, 1.2, 8, 48, path=path)
        assert not e["cached"]
        chosen = {kk: e[kk] for kk in autotune.KNOBS}
        assert pecann.get_tuning() == chosen
        assert e["build_ms"] <= e["rule_build_ms"] and e["knn_ms"] > 0
        stored = json.load(open(path))
        assert len(stored) == 1 and autotune.shape_key(ds, 24, 48, 8, 48) in stored
        pecann.reset_tuning()
        e2 = autotune.tune(ds, 24, 48, 1.2, 8, 48, path=path)
        assert e2["cached"] and pecann.get_tuning() == chosen
    finally:
        pecann.reset_tuning()


def test_tune_beam_meets_its_target_and_caches(tmp_path):
    dev = torch.device("cuda:0")
    X, _ = datagen.mixture(8000, 32, 12, seed=9)
    ds = pecann.Dataset(torch.from_numpy(X).to(dev), "l2", "f32")
    adj, deg = pecann.build_graph(ds, 32, 64, 1.2)
    path = str(tmp_path / "beam.json")
    e = autotune.tune_beam(ds, adj, deg, 10, target=0.97, path=path)
    assert not e["cached"] and 10 <= e["L_search"] <= 256
    if e["L_search"] < 256:
        assert e["agreement"] >= 0.97
        # every smaller beam that was tried fell short of the target
        assert all(t["agreement"] < 0.97 for t in e["tried"][:-1])
    # the chosen beam reproduces the measured agreement against the wide search
    ref = pecann.knn_density(ds, 10, adj, deg, L_search=256, rerank=256)[0].cpu().numpy()
    got = pecann.knn_density(ds, 10, adj, deg, L_search=e["L_search"], rerank=e["L_search"])[0].cpu().numpy()
    rows = np.arange(0, 8000, max(1, 8000 // 20000))[:20000]
    agree = np.mean([len(set(got[i]) & set(ref[i])) / 10 for i in rows])
    assert abs(agree - e["agreement"]) < 1e-6
    assert autotune.tune_beam(ds, adj, deg, 10, target=0.97, path=path)["cached"]
