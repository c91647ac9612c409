"""Build the HIP library libphx.so for gfx950 (in-tree), and the benchmark's probe library."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libphx.so")
SOURCES = ["phx_api.cpp", "phx_trace.hip", "phx_readout.hip", "phx_moments.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


# the benchmark's memory-system probe, a library of its own (not part of the trace)
PROBE_LIB = os.path.join(HERE, "libphx_probe.so")
PROBE_SOURCES = ["probe.hip"]


def _link(lib, sources, verbose):
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    _link(LIB, SOURCES, verbose)
    _link(PROBE_LIB, PROBE_SOURCES, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
