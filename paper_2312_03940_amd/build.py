"""Build libpecann.so (HIP, gfx950) in-tree.

    python -m paper_2312_03940_amd.build

Each .hip translation unit under csrc/ is compiled separately (in parallel) and
linked into paper_2312_03940_amd/libpecann.so.  Packed-FP32 VALU instructions are
disabled for all device code.  build(checked=True) makes the checked build,
libpecann_checked.so (-DPECANN_CHECKED: kernels test their invariants and the
entry points fail with PECANN_ECHECK when one breaks).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpecann.so")
LIB_CHECKED = os.path.join(PKG, "libpecann_checked.so")
BUILD_CHECKED = os.path.join(ROOT, "_build_checked")
ARCH = os.environ.get("PECANN_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, checked: bool = False) -> str:
    obj = os.path.join(BUILD_CHECKED if checked else BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *(["-DPECANN_CHECKED"] if checked else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True, jobs: int | None = None, checked: bool = False) -> str:
    os.makedirs(BUILD_CHECKED if checked else BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, checked), srcs))
    lib = LIB_CHECKED if checked else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True)
    build(verbose=True, checked=True)
    sys.exit(0)
