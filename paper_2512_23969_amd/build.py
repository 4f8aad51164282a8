"""Build the gfx950 shared library ``libslh.so`` in-tree with hipcc.

Usage: ``python -m paper_2512_23969_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libslh.so")
SOURCES = [os.path.join(CSRC, "api.hip"), os.path.join(CSRC, "serve.hip")]
# VALU issue-rate calibration program (the roofline's per-unit ceilings)
PROBE_SRC = os.path.join(CSRC, "valu_probe.hip")
PROBE = os.path.join(HERE, "valu_probe")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None) -> str:
    """Compile every HIP source into one shared library; returns its path."""
    out = out or LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + (extra or []) + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    if out == LIB:
        build_probe(verbose)
    return out


def build_probe(verbose: bool = False) -> str:
    """Compile the VALU calibration program (an executable, not part of the library)."""
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    tmp = PROBE + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + flags + [PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
