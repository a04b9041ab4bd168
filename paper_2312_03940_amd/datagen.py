"""Seeded synthetic workloads shaped like the paper's datasets.

This module is the only code that both the GPU path's tests/benchmark and the
CPU oracle consume.  It draws random numbers and lays out arrays; it holds none
of the method's arithmetic (no distances, densities, searches or clustering).

The generators follow the paper's "gaussian" recipe (Sec. 6.1, Datasets: centers
drawn uniformly from a box, then n/c points per center from an isotropic
Gaussian), at the shapes of its workloads.  The real datasets (MNIST, ImageNet
embeddings, ...) are not available; these stand in for them:

  config 1  10,000 x 16 float32, 10 centers ~ U[-10,10]^16, sigma = 1.
            An integer-grid twin (affine map to [0, 511], rounded) makes every
            float32 squared distance an exact integer.
  config 2  70,000 x 784 uint8 (MNIST-shaped): 10 centers ~ U[0,1]^784, variance
            0.05, 7,000 points each, then clip(round(255 x), 0, 255).
  config 3  1,000,000 x 128 float32: 1,000 centers ~ U[-10,10]^128 with per-cluster
            sigma ~ U[0.5, 2], 950 points each, plus 50,000 uniform background points.
  config 4  1,280,000 x 1024 float32 unit vectors (ImageNet-embedding-shaped):
            1,000 random unit centers u_c, x = normalize(u_c + s g), g ~ N(0, I),
            s = sqrt((1/0.49 - 1)/1024), so the mean cosine to the center is ~0.7.
  config 5  64 instances, n_i log-uniform in [2,000, 200,000], d = 384, 5..200
            centers ~ U[-10,10]^384, sigma = 1, k_i in {5, 10, 20}.

Every generator shuffles the points (index order carries no cluster
information) and returns the ground-truth component of each point.
Seeds: 20231203 + config number.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 20231203

# parameters of each configuration's workload (k, R, L, alpha, n_c, metric)
CONFIGS = {
    1: dict(n=10_000, d=16, k=10, n_c=10, metric="l2", dtype="f32"),
    2: dict(n=70_000, d=784, k=10, n_c=10, R=64, L=128, alpha=1.2, metric="l2", dtype="u8"),
    3: dict(n=1_000_000, d=128, k=16, n_c=1000, R=64, L=128, alpha=1.2, metric="l2",
            dtype="f32"),
    4: dict(n=1_280_000, d=1024, k=10, n_c=1000, R=64, L=200, alpha=1.2, metric="cosine",
            dtype="f32"),
    5: dict(instances=64, d=384, R=64, L=128, alpha=1.2, metric="l2", dtype="f32"),
}


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config + 1000 * salt)


def _shuffle(rng, X, y):
    p = rng.permutation(len(X))
    return np.ascontiguousarray(X[p]), np.ascontiguousarray(y[p])


def mixture(n: int, d: int, n_clusters: int, seed: int, box=(-10.0, 10.0), sigma=1.0,
            grid: int | None = None, dtype=np.float32):
    """Isotropic Gaussian mixture with equal cluster sizes (the last absorbs the remainder).

    grid=G maps the points affinely onto [0, G] and rounds them, so squared
    distances are exact integers in float32 whenever d * G^2 < 2^24.
    """
    rng = np.random.default_rng(seed)
    centers = rng.uniform(box[0], box[1], size=(n_clusters, d))
    sizes = np.full(n_clusters, n // n_clusters)
    sizes[-1] += n - sizes.sum()
    y = np.repeat(np.arange(n_clusters), sizes)
    X = centers[y] + sigma * rng.standard_normal((n, d))
    if grid is not None:
        lo, hi = X.min(), X.max()
        X = np.rint((X - lo) / (hi - lo) * grid)
    X, y = _shuffle(rng, X.astype(dtype), y)
    return X, y


def config1(integer_grid: bool = False):
    c = CONFIGS[1]
    X, y = mixture(c["n"], c["d"], 10, SEED_BASE + 1, grid=511 if integer_grid else None)
    return X, y


def config2(n: int | None = None):
    """MNIST-shaped uint8 mixture.  n < 70,000 gives a prefix-sized variant (same recipe)."""
    c = CONFIGS[2]
    n = c["n"] if n is None else n
    rng = rng_for(2)
    centers = rng.uniform(0.0, 1.0, size=(10, c["d"]))
    sizes = np.full(10, n // 10)
    sizes[-1] += n - sizes.sum()
    y = np.repeat(np.arange(10), sizes)
    X = np.empty((n, c["d"]), dtype=np.uint8)
    sd = np.sqrt(0.05)
    for s in range(0, n, 10_000):
        e = min(n, s + 10_000)
        blk = centers[y[s:e]] + sd * rng.standard_normal((e - s, c["d"]))
        X[s:e] = np.clip(np.rint(255.0 * blk), 0, 255).astype(np.uint8)
    return _shuffle(rng, X, y)


def config3(n_clusters: int = 1000, per_cluster: int = 950, background: int = 50_000):
    c = CONFIGS[3]
    d = c["d"]
    rng = rng_for(3)
    centers = rng.uniform(-10.0, 10.0, size=(n_clusters, d))
    sig = rng.uniform(0.5, 2.0, size=n_clusters)
    n = n_clusters * per_cluster + background
    X = np.empty((n, d), dtype=np.float32)
    y = np.empty(n, dtype=np.int64)
    for ci in range(n_clusters):
        s = ci * per_cluster
        X[s:s + per_cluster] = centers[ci] + sig[ci] * rng.standard_normal((per_cluster, d))
        y[s:s + per_cluster] = ci
    s = n_clusters * per_cluster
    X[s:] = rng.uniform(-10.0, 10.0, size=(background, d))
    y[s:] = -1  # background noise has no component
    return _shuffle(rng, X, y)


def config4(n_clusters: int = 1000, per_cluster: int = 1280, d: int = 1024):
    rng = rng_for(4)
    u = rng.standard_normal((n_clusters, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    s = np.sqrt((1.0 / 0.49 - 1.0) / d)
    n = n_clusters * per_cluster
    X = np.empty((n, d), dtype=np.float32)
    y = np.repeat(np.arange(n_clusters), per_cluster)
    for ci in range(n_clusters):
        blk = u[ci] + s * rng.standard_normal((per_cluster, d))
        blk /= np.linalg.norm(blk, axis=1, keepdims=True)
        X[ci * per_cluster:(ci + 1) * per_cluster] = blk
    return _shuffle(rng, X, y)


def config5_instances(count: int = 64, n_lo: int = 2_000, n_hi: int = 200_000):
    """Per-instance (n_i, n_clusters_i, k_i, seed_i) of the batched workload."""
    rng = rng_for(5)
    n = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count)).astype(np.int64)
    ncl = rng.integers(5, 201, size=count)
    k = rng.choice(np.array([5, 10, 20]), size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [dict(n=int(n[i]), n_clusters=int(ncl[i]), k=int(k[i]), seed=int(seeds[i]))
            for i in range(count)]


def config5_instance(spec: dict, d: int = 384):
    return mixture(spec["n"], d, spec["n_clusters"], spec["seed"])


def config5(count: int = 64, d: int = 384):
    """Every instance of the batched workload, stacked in instance order.

    -> (X float32 [N, d], y int64 [N] (component ids, distinct across instances),
        offsets int64 [count + 1], k int32 [count], n_clusters int32 [count])."""
    specs = config5_instances(count)
    sizes = np.array([sp["n"] for sp in specs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = np.empty((int(off[-1]), d), dtype=np.float32)
    y = np.empty(int(off[-1]), dtype=np.int64)
    base = 0
    for t, sp in enumerate(specs):
        Xt, yt = config5_instance(sp, d)
        X[off[t]:off[t + 1]] = Xt
        y[off[t]:off[t + 1]] = yt + base
        base += sp["n_clusters"]
    k = np.array([sp["k"] for sp in specs], dtype=np.int32)
    ncl = np.array([sp["n_clusters"] for sp in specs], dtype=np.int32)
    return X, y, off, k, ncl


def permutation(n: int, seed: int) -> np.ndarray:
    """Insertion order for the batched graph build (int32)."""
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


def random_neighbour_lists(n: int, K: int, seed: int, repeats: int = 1) -> np.ndarray:
    """Random starting lists for an NN-descent construction: for each repeat and
    each point i, K distinct ids drawn uniformly from the other n - 1 points
    (Floyd's sampling, vectorised over points).  -> int32 [repeats, n, K]."""
    if not 1 <= K <= n - 1:
        raise ValueError("need 1 <= K <= n - 1")
    rng = np.random.default_rng(seed)
    out = np.empty((repeats, n, K), dtype=np.int32)
    rows = np.arange(n, dtype=np.int64)
    N = n - 1
    for r in range(repeats):
        S = np.empty((n, K), dtype=np.int64)
        for c, j in enumerate(range(N - K, N)):
            t = rng.integers(0, j + 1, size=n, dtype=np.int64)
            taken = (S[:, :c] == t[:, None]).any(axis=1) if c else np.zeros(n, bool)
            S[:, c] = np.where(taken, j, t)
        out[r] = (S + (S >= rows[:, None])).astype(np.int32)  # skip the row's own index
    return out
