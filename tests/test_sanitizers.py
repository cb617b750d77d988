"""The FP64 oracle and libseb's host code built with the address and
undefined-behaviour sanitizers (host code only: the kernel launchers and the
HIP runtime calls are host stand-ins, tests/sanitize/host_stubs.cpp) and run
over their entry points on small seeded inputs: any out-of-bounds access,
use after free, leak or undefined operation fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.slow


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", *SAN, "-I", os.path.join(ROOT, "oracle"),
         os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
    r = run([exe], env=dict(ENV, OMP_NUM_THREADS="2"))
    assert "oracle driver ok" in r.stdout
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


def clang():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++"),
              shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(clang() is None, reason="clang++ not available")
def test_host_library_under_sanitizers(tmp_path):
    cxx = clang()
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2503_02412_amd", "csrc"),
           "-I", os.path.join(rocm, "include"), "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src in (os.path.join(ROOT, "paper_2503_02412_amd", "csrc", "seb_host.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_stubs.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        run([cxx, "-x", "c++", "-std=c++17", "-ffp-contract=off", *SAN, *inc, "-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    run([cxx, *SAN, *objs, "-o", exe])
    r = run([exe], env=ENV)
    assert "host driver ok" in r.stdout
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
