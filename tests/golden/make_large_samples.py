"""Writes tests/golden/c3_sample.npz, c4_sample.npz and c5_sample.npz: the
oracle's exact neighbours of a fixed 2,000-point sample of the 1,000,000 x 128
mixture (k = 16, L2), of the 1,280,000 x 1024 unit-vector mixture (k = 10,
cosine) and of the 64-instance batch (each point within its own instance, with
its instance's k; rows padded to 20 with +inf).  Used by the recall@k gates of
bench.py --config 3 / 4 / 5.  Calls only the oracle and the seeded generator:

    python tests/golden/make_large_samples.py [3] [4] [5]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2312_03940_amd import datagen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_ids(n, count=2000):
    return np.arange(0, n, n // count)[:count].astype(np.int64)


def run5():
    t = time.time()
    X, _, off, k, _ = datagen.config5()
    n = X.shape[0]
    q = sample_ids(n)
    kmax = int(k.max())
    dist = np.full((len(q), kmax), np.inf)
    idx = np.full((len(q), kmax), -1, dtype=np.int64)
    qk = np.zeros(len(q), dtype=np.int32)
    inst = np.searchsorted(off, q, side="right") - 1
    for ti in np.unique(inst):
        lo, hi = int(off[ti]), int(off[ti + 1])
        rows = np.nonzero(inst == ti)[0]
        P = oracle.Points(X[lo:hi], oracle.L2)
        ii, dd = oracle.knn(P, int(k[ti]), q[rows] - lo)
        idx[rows, :k[ti]] = ii + lo
        dist[rows, :k[ti]] = dd
        qk[rows] = k[ti]
    out = os.path.join(HERE, "c5_sample.npz")
    np.savez_compressed(out, sample=q.astype(np.int32), knn_idx=idx.astype(np.int32), knn_dist=dist,
                        k=qk)
    print(f"wrote {out} in {time.time() - t:.1f} s (oracle threads {oracle.num_threads()})")


def run(cfg):
    if cfg == 5:
        return run5()
    t = time.time()
    if cfg == 3:
        X, _ = datagen.config3()
        metric, k = oracle.L2, datagen.CONFIGS[3]["k"]
    else:
        X, _ = datagen.config4()
        metric, k = oracle.COSINE, datagen.CONFIGS[4]["k"]
    P = oracle.Points(X, metric)
    q = sample_ids(X.shape[0])
    idx, dist = oracle.knn(P, k, q)
    out = os.path.join(HERE, f"c{cfg}_sample.npz")
    np.savez_compressed(out, sample=q.astype(np.int32), knn_idx=idx.astype(np.int32),
                        knn_dist=dist, k=np.int32(k))
    print(f"wrote {out} in {time.time() - t:.1f} s (oracle threads {oracle.num_threads()})")


if __name__ == "__main__":
    for c in (sys.argv[1:] or ["3", "4"]):
        run(int(c))
