"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard and the
workload table the GPU tests and the benchmark share."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_workload_table_matches_the_benchmark_configurations():
    # the headline is the largest single-GPU workload (1.28M x 1024 cosine, FP8
    # rows with a float32 rerank); the MNIST-shaped one runs float32 rows
    wl = bench.WORKLOADS
    assert set(wl) == {2, 3, 4, 5}
    assert (wl[2]["search"], wl[2]["R"], wl[2]["L"], wl[2]["alpha"], wl[2]["k"], wl[2]["n_c"]) == \
        ("f32", 64, 128, 1.2, 10, 10)
    assert (wl[3]["search"], wl[3]["R"], wl[3]["L"], wl[3]["k"], wl[3]["n_c"]) == ("bf16", 64, 128, 16, 1000)
    assert (wl[4]["search"], wl[4]["metric"], wl[4]["R"], wl[4]["L"], wl[4]["k"]) == ("fp8", "cosine", 64, 200, 10)
    assert wl[5]["search"] == "bf16" and wl[5]["n_c"] is None
    sys_argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        args = bench.parse()
    finally:
        sys.argv = sys_argv
    assert args.gpus == 1 and args.config == 4
