"""Builds the native parts in-tree (no GPU needed: hipcc cross-compiles gfx950).

  liblprdem.so   HIP kernels + C ABI (include/lprdem.h), gfx950
  libbedgen.so   seeded bed generator (plain C)
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HIP_SOURCES = ["lpr_kernels.hip", "lpr_adjoint.hip", "lpr_spook.hip", "lpr_runtime.hip"]


def _run(cmd, verbose):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    if verbose and (r.stdout or r.stderr):
        print(r.stdout + r.stderr)


def build_lprdem(verbose=False) -> str:
    out = os.path.join(HERE, "liblprdem.so")
    cmd = [HIPCC, *HIP_FLAGS, "-I" + os.path.join(ROOT, "include"),
           *[os.path.join(CSRC, s) for s in HIP_SOURCES], "-o", out + ".tmp"]
    _run(cmd, verbose)
    os.replace(out + ".tmp", out)
    return out


def build_bedgen(verbose=False) -> str:
    out = os.path.join(HERE, "libbedgen.so")
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-Wall", os.path.join(CSRC, "bedgen.c"), "-o", out + ".tmp", "-lm"]
    _run(cmd, verbose)
    os.replace(out + ".tmp", out)
    return out


def build_all(verbose=False):
    return [build_bedgen(verbose), build_lprdem(verbose)]


if __name__ == "__main__":
    for p in build_all(verbose=True):
        print(p)
