"""The checked build (libpecann_checked.so, compiled with -DPECANN_CHECKED):
every kernel tests invariants of its inputs and state (item and neighbour ids
inside the point set, degrees at most R, the beam sorted and within its
capacity, a point inside the instance found for it, prune outputs within R,
light reverse targets within the LDS capacity, reverse edges inside the batch's
segments, kept exact-mode candidates and cluster labels in range) and an entry
point fails with PECANN_ECHECK when one breaks.  A child process loads the
checked library and runs the graph, doubling-round, exact-mode and reduced
precision parity tests against it: they must pass unchanged."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2312_03940_amd", "libpecann_checked.so")


@pytest.mark.gpu
def test_parity_under_the_checked_build():
    assert os.path.exists(LIB), "libpecann_checked.so is not built (run __graft_entry__.build())"
    env = dict(os.environ)
    env["PECANN_LIB"] = LIB
    sel = ("worked_example or integer_grid or bit_exact or threshold or isolated or "
           "mnist_shaped or c3_shaped or c4_shaped")
    r = subprocess.run([sys.executable, "-u", "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "gpu",
                        os.path.join(ROOT, "tests", "test_gpu_parity.py"), "-k", sel],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    out = r.stdout + r.stderr
    assert "device invariant check failed" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out


_BAD_GRAPH = r"""
import numpy as np, torch
from paper_2312_03940_amd import pecann
rng = np.random.default_rng(3)
n, d, R = 500, 8, 8
X = torch.from_numpy(rng.standard_normal((n, d)).astype(np.float32)).cuda()
ds = pecann.Dataset(X, "l2", "f32")
adj = rng.integers(0, n, (n, R)).astype(np.int32)
adj[7, 3] = n + 5  # outside the point set: the search skips it, the checked build reports it
deg = np.full(n, R, np.int32)
try:
    pecann.knn_density(ds, 5, torch.from_numpy(adj).cuda(), torch.from_numpy(deg).cuda(), L_search=16)
    torch.cuda.synchronize()
    print("RESULT ok")
except pecann.PecannError as e:
    print("RESULT error", e)
"""


@pytest.mark.gpu
def test_checked_build_reports_a_neighbour_outside_the_point_set():
    # a graph entry >= n is skipped by the search (never dereferenced): the
    # normal build returns results, the checked build fails the call
    out = {}
    for name, lib in (("normal", None), ("checked", LIB)):
        env = dict(os.environ)
        if lib:
            env["PECANN_LIB"] = lib
        r = subprocess.run([sys.executable, "-c", _BAD_GRAPH], capture_output=True, text=True, env=env,
                           cwd=ROOT, timeout=300)
        assert r.returncode == 0, r.stderr[-3000:]
        out[name] = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT")][-1]
    assert out["normal"] == "RESULT ok"
    assert "device invariant check failed" in out["checked"] and "0x2" in out["checked"], out["checked"]
