"""Builds ``librgg.so`` in-tree for gfx950.

* ``geometry.cpp`` (host build stage, binary64 with the C library's sin, cos,
  acos, sqrt) is compiled by g++ with FMA contraction and builtin folding off,
  so the approximations are exactly the stated binary64 expressions;
* ``api.cpp`` (C ABI, host side), ``server.cpp`` (request server),
  ``kernels.hip`` (update kernels) and ``validate.hip`` (full validation) by
  hipcc,
  device code with ``-ffp-contract=off`` so binary64 re-tests evaluate the same
  expressions, and with packed FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "librgg.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("RGG_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", f"-I{INC}", f"-I{CSRC}"]
    geo = os.path.join(BUILD, "geometry.o")
    api = os.path.join(BUILD, "api.o")
    ker = os.path.join(BUILD, "kernels.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin",
          "-Wall", f"-I{INC}", f"-I{CSRC}", "-c", os.path.join(CSRC, "geometry.cpp"), "-o", geo], verbose)
    _run([hipcc, *common, "-Wall", "-c", os.path.join(CSRC, "api.cpp"), "-o", api], verbose)
    srv = os.path.join(BUILD, "server.o")
    _run([hipcc, *common, "-Wall", "-c", os.path.join(CSRC, "server.cpp"), "-o", srv], verbose)
    _run([hipcc, *common, f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-c", os.path.join(CSRC, "kernels.hip"), "-o", ker], verbose)
    val = os.path.join(BUILD, "validate.o")
    _run([hipcc, *common, f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-c", os.path.join(CSRC, "validate.hip"), "-o", val], verbose)
    tmp = OUT + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, geo, api, srv, ker, val, "-lpthread"],
         verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
