"""Compile the HIP library (libhsm.so, gfx950) and the node generator in place.

Every HIP source is built with -ffp-contract=off (products and sums rounded as
written; FMAs are explicit where wanted) and without packed FP32 instructions.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhsm.so")
NODEGEN_SRC = os.path.join(PKG, "nodegen", "nodegen.c")
NODEGEN_LIB = os.path.join(PKG, "nodegen", "libhsm_nodegen.so")
SOURCES = ["abi.hip", "scan.hip", "build.hip", "solve.hip", "apply.hip", "sim.hip"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-pass-failed"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + out)
    return out


def build_nodegen():
    _run(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", NODEGEN_SRC, "-o", NODEGEN_LIB, "-lm"])
    return NODEGEN_LIB


def build_hip(jobs: int = 8, verbose: bool = False):
    os.makedirs(BUILD, exist_ok=True)
    objs = []

    def one(src):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        out = _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        if verbose and out.strip():
            print(out, file=sys.stderr)
        return obj

    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs])
    shutil.move(tmp, LIB)
    return LIB


def build_all(jobs: int = 8, verbose: bool = False):
    build_nodegen()
    return build_hip(jobs=jobs, verbose=verbose)


if __name__ == "__main__":
    print(build_all(verbose=True))
