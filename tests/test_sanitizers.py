"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, no GPU): the oracle is rebuilt with both sanitizers into a
temporary library, and its pin tests run against that build in a child
process with the sanitizer runtime preloaded.  Any out-of-bounds access,
use-after-free or undefined operation in the oracle aborts the child with a
sanitizer report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dpc_oracle.c")


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's AddressSanitizer runtime is not installed")
def test_oracle_pins_under_address_and_ub_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                    "-Wall", "-o", lib, SRC, "-lm"], check=True)
    env = dict(os.environ)
    env["PECANN_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = _runtime("libasan.so")
    # the interpreter itself is not instrumented: leak checks would report it
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_vamana_pins.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]


def _clang_asan():
    from paper_2312_03940_amd import build as B
    p = subprocess.run([B.HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_clang_asan() is None, reason="clang's AddressSanitizer runtime is not installed")
def test_abi_host_code_under_address_sanitizer(tmp_path):
    # the C ABI's host code (argument checks, layouts, workspace carving, tuning
    # state, error strings) built with AddressSanitizer (host side only: the
    # device code is compiled as usual) and linked with the other objects of
    # the in-tree build; the ABI tests then run against it in a child process
    from paper_2312_03940_amd import build as B
    objs = [os.path.join(B.BUILD, os.path.basename(s) + ".o") for s in B.sources()]
    if not all(os.path.exists(o) for o in objs):
        B.build(verbose=False)
    abi = os.path.join(B.CSRC, "pecann_abi.hip")
    obj = str(tmp_path / "pecann_abi_asan.o")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([B.HIPCC, *B.FLAGS, *san, "-g", "-c", abi, "-o", obj], check=True)
    lib = str(tmp_path / "libpecann_asan.so")
    others = [o for o in objs if not o.endswith("pecann_abi.hip.o")]
    subprocess.run([B.HIPCC, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *san, "-o", lib, obj, *others],
                   check=True)
    env = dict(os.environ)
    env["PECANN_LIB"] = lib
    env["LD_PRELOAD"] = _clang_asan()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
