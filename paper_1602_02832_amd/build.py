"""Compile the native libraries in-tree.

  libhtree.so       HIP kernels + C-ABI (include/htree.h: force path, integration;
                    include/htree_tree.h: tree and lists on the device), gfx950 only
  libhtree_host.so  host tree/list builder and Hermite corrector (include/htree_host.h)

Run ``python -m paper_1602_02832_amd.build``.  Every call recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

DEVICE_LIB = os.path.join(PKG, "libhtree.so")
HOST_LIB = os.path.join(PKG, "libhtree_host.so")

# packed FP32 instructions are never generated (build policy for this device)
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{INCLUDE}"]
DEVICE_SOURCES = ["htree.hip", "devtree.hip"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall", f"-I{INCLUDE}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_device(verbose: bool = False) -> str:
    """Compile the device sources in parallel, then link them into one library."""
    objs, procs = [], []
    for src in DEVICE_SOURCES:
        obj = os.path.join(PKG, "_obj_" + src.replace(".hip", ".o"))
        cmd = [HIPCC, *HIP_FLAGS, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append((cmd, subprocess.Popen(cmd)))
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = DEVICE_LIB + ".tmp"
    try:
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    os.replace(tmp, DEVICE_LIB)
    return DEVICE_LIB


def build_host(verbose: bool = False) -> str:
    tmp = HOST_LIB + ".tmp"
    _run(["g++", *HOST_FLAGS, "-o", tmp, os.path.join(CSRC, "hosttree.cpp")], verbose)
    os.replace(tmp, HOST_LIB)
    return HOST_LIB


def build(verbose: bool = False) -> None:
    build_host(verbose)
    build_device(verbose)


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
