"""Builds the native parts of the package in-tree:

* ``libpacim.so``               the HIP library (gfx950) behind include/pacim.h
* ``inputs/libpacim_gen.so``    the seeded graph generators (host C)

Run as ``python -m paper_2311_07554_amd.build_native`` or through
``__graft_entry__.build()``.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PACIM_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed FP32 instructions out of every code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build_hip():
    out = os.path.join(PKG, "libpacim.so")
    tmp = out + ".tmp"
    _run([HIPCC, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
          "-o", tmp, os.path.join(PKG, "csrc", "pacim.hip")])
    os.replace(tmp, out)
    return out


def build_gen():
    out = os.path.join(PKG, "inputs", "libpacim_gen.so")
    _run(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", out,
          os.path.join(PKG, "inputs", "graphgen.c"), "-lm"])
    return out


def build_all():
    build_gen()
    build_hip()


if __name__ == "__main__":
    build_all()
    sys.exit(0)
