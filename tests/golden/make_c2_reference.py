"""Writes tests/golden/c2_reference.npz: the oracle's exact DPC of the MNIST-shaped
workload (70,000 x 784 uint8, k = 10, n_c = 10, product centers), used by the
benchmark's quality gates (ARI vs the oracle, recall@10) and by the full-size GPU
parity test.  It calls only the oracle and the seeded generator:

    python tests/golden/make_c2_reference.py

Stored: labels (int32 root index per point), rank (int32 density rank), dep (int32
exact dependent point, -1 for the densest), and for a fixed sample of 2,000 query
points their exact 10-NN indices and distances.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2312_03940_amd import datagen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_reference.npz")


def main():
    t = time.time()
    X, _ = datagen.config2()
    k, n_c = datagen.CONFIGS[2]["k"], datagen.CONFIGS[2]["n_c"]
    ref = oracle.exact_dpc(X, k=k, n_c=n_c)
    sample = np.arange(0, X.shape[0], X.shape[0] // 2000)[:2000].astype(np.int32)
    np.savez_compressed(OUT, labels=ref["labels"].astype(np.int32),
                        rank=ref["rank"].astype(np.int32), dep=ref["dep"].astype(np.int32),
                        sample=sample,
                        sample_knn_idx=ref["knn_idx"][sample].astype(np.int32),
                        sample_knn_dist=ref["knn_dist"][sample],
                        k=np.int32(k), n_c=np.int32(n_c))
    print(f"wrote {OUT} in {time.time() - t:.1f} s "
          f"({len(np.unique(ref['labels']))} clusters, oracle threads {oracle.num_threads()})")


if __name__ == "__main__":
    main()
