"""Benchmark of the DPC hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (the MNIST-shaped configuration): 70,000 x 784 uint8 points from a seeded
10-Gaussian mixture scaled into [0, 255], L2 distance, float32 search rows, Vamana
graph with R = 64, build beam L = 128, alpha = 1.2 (two passes), kth density with
k = 10, doubling dependent search (L_d = 64, threshold = 300), 10 product centers.

One step = the whole hot path on resident data: prepare_vectors -> build_graph ->
knn_density -> dependent_search -> cluster, all on one HIP stream.  `value` is DPC
points/s = n * K / (time of K steps).  Quality gates after timing: ARI of the
labels against the oracle's exact DPC, and recall@10 of the kNN on a 2,000-query
sample, both from tests/golden/c2_reference.npz (written by the oracle).

`roofline` reports the kNN search launch (search_kernel<f32, 16, MODE_KNN>, the
single largest gather-bound launch): algorithmic bytes from the kernel's own work
counters divided by its HIP-event time; `cpu_baseline` times the CPU oracle's
exact DPC on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DPC points/s at ARI>=0.95 vs oracle; kNN queries/s at recall@10>=0.95"
HBM_PEAK_GBS = 8000.0
REF_PATH = os.path.join(ROOT, "tests", "golden", "c2_reference.npz")
TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic.json")


def stored_traffic(key: str):
    """HBM bytes per launch measured by the FETCH_SIZE/WRITE_SIZE runs, or None when
    missing or when the search kernel's sources changed since they were taken."""
    from paper_2312_03940_amd.kernel_hash import search_kernel_hash
    if not os.path.exists(TRAFFIC_PATH):
        return None
    with open(TRAFFIC_PATH) as f:
        t = json.load(f)
    if t.get("source_hash") != search_kernel_hash() or key not in t:
        return None
    return int(t[key]["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--search", default="f32", choices=["f32", "u8"])
    ap.add_argument("--L-search", type=int, default=64)
    ap.add_argument("--L-d", type=int, default=64)
    ap.add_argument("--threshold", type=int, default=300)
    ap.add_argument("--kdep-cap", type=int, default=1024)
    ap.add_argument("--num-starts", type=int, default=8)
    ap.add_argument("--max-batch", type=int, default=0,
                    help="build batch cap (0: the library default, max(n/50, 8192))")
    ap.add_argument("--cpu-sample", type=int, default=16000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a reference "
                         "kernel of known traffic for hardware byte counters)")
    return ap.parse_args()


def ari(a, b) -> float:
    from sklearn.metrics import adjusted_rand_score
    return float(adjusted_rand_score(a, b))


def cpu_baseline(X, ref, sample_size):
    """The oracle as it stands: exact kNN (k = 10) and exact dependent points of a
    sample of points against all n points, FP64, all host threads."""
    import oracle
    P = oracle.Points(X)
    n = X.shape[0]
    q = np.linspace(0, n - 1, sample_size).astype(np.int64)
    rank = ref["rank"].astype(np.int64)
    t0 = time.perf_counter()
    oracle.knn(P, 10, q)
    oracle.dependent_exact(P, rank, q)
    dt = time.perf_counter() - t0
    return {"value": sample_size / dt, "unit": "points/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": (f"exact DPC (FP64 brute-force 10-NN + Def. 1 dependent) of "
                                         f"{sample_size} evenly spaced points against all {n}; "
                                         f"density ranks from the stored oracle run"),
            "seconds": dt}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2312_03940_amd import datagen, pecann

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cfg = datagen.CONFIGS[2]
    R, L, alpha, k, n_c = cfg["R"], cfg["L"], cfg["alpha"], cfg["k"], cfg["n_c"]

    X, _ = datagen.config2()
    n, d = X.shape
    perm_h = datagen.permutation(n, 20231205)
    x = torch.from_numpy(X).to(dev)
    perm = torch.from_numpy(perm_h).to(dev)
    ds = pecann.Dataset(x, "l2", args.search)

    # every buffer of the step is allocated here, outside the timed region
    wsb = pecann.workspace_bytes(ds, k, args.L_search, args.kdep_cap, R, L, alpha, args.num_starts,
                                 args.max_batch)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    g_out = (torch.empty((n, R), dtype=torch.int32, device=dev),
             torch.empty(n, dtype=torch.int32, device=dev))
    k_out = (torch.empty((n, k), dtype=torch.int32, device=dev),
             torch.empty((n, k), dtype=torch.float32, device=dev),
             torch.empty(n, dtype=torch.float32, device=dev),
             torch.empty(n, dtype=torch.int64, device=dev))
    d_out = (torch.empty(n, dtype=torch.int32, device=dev),
             torch.empty(n, dtype=torch.float32, device=dev),
             torch.zeros(32, dtype=torch.int32, device=dev))
    c_out = (torch.empty(n, dtype=torch.int32, device=dev),
             torch.empty(n, dtype=torch.uint8, device=dev))
    phases = ["prepare", "build", "knn_density", "dependent", "cluster"]

    def step(events=None, bcnt=None, kcnt=None):
        ev = events
        if ev:
            ev[0].record()
        ds.prepare(x)
        if ev:
            ev[1].record()
        adj, deg = pecann.build_graph(ds, R, L, alpha, num_starts=args.num_starts, perm=perm,
                                      max_batch=args.max_batch, ws=ws, out=g_out, counters=bcnt)
        if ev:
            ev[2].record()
        idx, dist, rho, key = pecann.knn_density(ds, k, adj, deg, L_search=args.L_search, ws=ws,
                                                 out=k_out, counters=kcnt)
        if ev:
            ev[3].record()
        dep, delta, stats = pecann.dependent_search(ds, key, idx, dist, adj, deg, L_d=args.L_d,
                                                    L_search=args.L_search,
                                                    threshold=args.threshold,
                                                    kdep_cap=args.kdep_cap, ws=ws, out=d_out)
        if ev:
            ev[4].record()
        pecann.cluster(rho, dep, delta, n_c=n_c, ws=ws, out=c_out)
        if ev:
            ev[5].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.copy_probe_mb:
        src = torch.empty(args.copy_probe_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    pecann.profile_enable(True)  # per-kernel HIP events on the launch stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pecann.profile_enable(False)
    kprof = pecann.profile_report()

    ph = {p: [] for p in phases}
    for e in evs:
        for j, p in enumerate(phases):
            ph[p].append(e[j].elapsed_time(e[j + 1]))
    ms_per_step = wall * 1e3 / args.steps
    value = n * args.steps / wall
    knn_ms = float(np.median(ph["knn_density"]))


    # work counters from one extra (untimed) step
    bcnt = torch.zeros(8, dtype=torch.int64, device=dev)
    kcnt = torch.zeros(4, dtype=torch.int64, device=dev)
    step(bcnt=bcnt, kcnt=kcnt)
    torch.cuda.synchronize()
    bc = bcnt.cpu().numpy().astype(np.int64)
    kc = kcnt.cpu().numpy().astype(np.int64)

    # quality gates
    quality = {}
    ref = None
    if os.path.exists(REF_PATH):
        ref = np.load(REF_PATH)
        labels = c_out[0].cpu().numpy()
        quality["ari_vs_oracle"] = ari(labels, ref["labels"])
        s = ref["sample"]
        gi = k_out[0].cpu().numpy()[s]
        gd = k_out[1].cpu().numpy()[s]
        thr = ref["sample_knn_dist"][:, k - 1]
        # a returned point counts when its distance (exact here: integer rows) is within the
        # oracle's k-th distance; duplicates and the query itself never count
        hits = 0
        for t in range(len(s)):
            seen = set()
            for j, dj in zip(gi[t], gd[t]):
                if j < 0 or j == s[t] or j in seen:
                    continue
                seen.add(int(j))
                hits += float(dj) <= np.float32(thr[t])
        quality["recall_at_10"] = hits / (k * len(s))
        quality["gates_met"] = bool(quality["ari_vs_oracle"] >= 0.95 and quality["recall_at_10"] >= 0.95)
    else:
        quality["missing"] = "tests/golden/c2_reference.npz not found"

    row_bytes = {"f32": 4 * d, "u8": d}[args.search]
    # algorithmic bytes per step of each gather kernel family, from its own counters:
    # per expansion the degree word and the neighbour ids, per distance the candidate
    # row, per search its own row and its outputs
    nsearch_build = 2 * n - 1
    alg = {
        "search_knn": 4 * (kc[0] + kc[1]) + row_bytes * kc[2] + n * row_bytes + n * (k * 8 + 4 + 8),
        "search_build": (4 * (bc[0] + bc[1]) + row_bytes * bc[2] + nsearch_build * row_bytes
                         + 8 * bc[0] + 4 * nsearch_build),
    }
    fam_ms = {f: v[1] / args.steps for f, v in kprof.items()}
    fam_launch = {f: v[0] / args.steps for f, v in kprof.items()}
    dom = max(fam_ms, key=fam_ms.get)
    rl_fam = dom if dom in alg else max(alg, key=lambda f: fam_ms.get(f, 0.0))
    avg_launch_ms = fam_ms[rl_fam] / fam_launch[rl_fam]
    bytes_per_launch = alg[rl_fam] / fam_launch[rl_fam]
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    knl = {"search_build": "MODE_BUILD", "search_knn": "MODE_KNN"}[rl_fam]
    roofline = {"bound": "hbm", "kernel": f"search_kernel<{args.search}, G=16, {knl}>",
                "family": rl_fam, "dominant_family": dom,
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic(f"{rl_fam}@{args.search}"),
                "alg_bytes_per_launch": int(bytes_per_launch),
                "avg_launch_ms": round(avg_launch_ms, 4), "launches_per_step": fam_launch[rl_fam],
                "knn_launch": {"ms": round(fam_ms.get("search_knn", 0.0), 3),
                               "achieved_GBps": round(alg["search_knn"] / (fam_ms["search_knn"] * 1e-3) / 1e9, 1)
                               if "search_knn" in fam_ms else None,
                               "per_query": {"expansions": kc[0] / n, "ids_read": kc[1] / n,
                                             "rows_gathered": kc[2] / n}}}
    kernels_ms = {f: {"launches_per_step": fam_launch[f], "ms_per_step": round(v, 3)}
                  for f, v in sorted(fam_ms.items(), key=lambda t: -t[1])}

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.search, "data": "synthetic",
        "config": {"workload": "MNIST-shaped 70000x784 uint8 10-Gaussian mixture, L2",
                   "n": n, "d": d, "search_rows": args.search, "R": R, "L_build": L,
                   "alpha": alpha, "build_passes": 2, "num_starts": args.num_starts,
                   "max_batch": args.max_batch or max(n // 50, 8192),
                   "k": k, "L_search": args.L_search, "L_d": args.L_d,
                   "threshold": args.threshold, "kdep_cap": args.kdep_cap, "n_c": n_c,
                   "parallelism": "single GPU"},
        "knn_queries_per_s": round(n / (knn_ms * 1e-3), 1),
        "phases_ms": {p: round(float(np.median(v)), 3) for p, v in ph.items()},
        "quality": quality,
        "build_work": {"search_expansions": int(bc[0]), "search_rows": int(bc[2]),
                       "forward_prune_rows": int(bc[4]), "reverse_prune_rows": int(bc[5]),
                       "targets_pruned": int(bc[6]), "targets_appended": int(bc[7])},
        "dependent_stats": d_out[2].cpu().numpy()[:8].tolist(),
        "kernels_ms": kernels_ms,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline and ref is not None:
        out["cpu_baseline"] = cpu_baseline(X, ref, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
