"""Compile the HIP library (libseb.so) for gfx950, in-tree.

    python -m paper_2503_02412_amd.build

Host code is compiled without floating-point contraction so that its FP64
footprint table is computed exactly as written.  Device code is compiled with
packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libseb.so")
ARCH = os.environ.get("SEB_OFFLOAD_ARCH", "gfx950")

HOST_SOURCES = ["seb_host.cpp"]
DEVICE_SOURCES = ["seb_assess.hip", "seb_net.hip", "seb_surrogate.hip", "seb_sdf.hip",
                  "seb_elevation.hip"]

COMMON = ["-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{ROOT}/include"]
# Code-object v5 loads under every ROCm 6.x/7.x runtime, including the HIP
# runtime bundled with the PyTorch wheel (which the library binds to when torch
# is imported first: both carry the SONAME libamdhip64.so.7).
DEVICE_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-Xclang",
                "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _rocm() -> str:
    return os.environ.get("ROCM_PATH", "/opt/rocm")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    return r


def build_library(verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([hipcc, "-x", "c++", *COMMON, *HOST_FLAGS, "-D__HIP_PLATFORM_AMD__",
              f"-I{_rocm()}/include",
              "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in DEVICE_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([hipcc, *COMMON, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5", *objs,
          "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
