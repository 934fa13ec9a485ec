"""Compile the HIP library libifmm.so for gfx950, in-tree.

The library is one translation unit (csrc/ifmm.hip, which includes the other
sources). hipcc cross-compiles without a GPU.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "ifmm.hip")
OUT = os.path.join(HERE, "libifmm.so")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    cmd = [hipcc] + FLAGS + [SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for %s" % SRC)
    os.replace(tmp, OUT)
    return OUT


HOST_SRC = os.path.join(ROOT, "tests", "host", "host_checks.cpp")
HOST_OUT = os.path.join(ROOT, "tests", "host", "host_checks")


def build_host_checks(verbose: bool = False) -> str:
    """The host-only check program of the planning logic (tests/host)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-x", "hip", "-Wno-unused-result",
           "-I" + os.path.join(ROOT, "include"), HOST_SRC, "-o", HOST_OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for %s" % HOST_SRC)
    os.replace(HOST_OUT + ".tmp", HOST_OUT)
    return HOST_OUT


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_host_checks(verbose=True))
