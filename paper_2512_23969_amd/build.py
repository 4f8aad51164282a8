"""Build the gfx950 shared library ``libslh.so`` in-tree with hipcc.

The host code of each parameter set, with the kernels it instantiates, is
its own translation unit (``csrc/set_<id>.hip``); the units compile in
parallel into ``_build/`` and are linked into one library.

Usage: ``python -m paper_2512_23969_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libslh.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ([os.path.join(CSRC, "api.hip"), os.path.join(CSRC, "serve.hip")]
           + sorted(glob.glob(os.path.join(CSRC, "set_*.hip"))))
# VALU issue-rate calibration program (the roofline's per-unit ceilings)
PROBE_SRC = os.path.join(CSRC, "valu_probe.hip")
PROBE = os.path.join(HERE, "valu_probe")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _compile(src: str, extra: list[str], verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    tmp = obj + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + (extra or []) + ["-c", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, obj)
    return obj


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None) -> str:
    """Compile every HIP source (in parallel) and link one shared library;
    returns its path."""
    out = out or LIB
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(_jobs()) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra or [], verbose), SOURCES))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    if out == LIB:
        build_probe(verbose)
    return out


def build_probe(verbose: bool = False) -> str:
    """Compile the VALU calibration program (an executable, not part of the library)."""
    flags = [f for f in FLAGS if f != "-fPIC"]
    tmp = PROBE + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + flags + [PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
