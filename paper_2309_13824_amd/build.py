"""Builds libtrime.so (HIP for gfx950) in the package directory.

hipcc compiles the kernels for gfx950 only.  Floating-point contraction is
off (the kernels request FMA explicitly where they want it) and the packed
FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtrime.so")
SOURCES = ["persist.hip", "cells.hip", "abi.hip", "adapt.hip", "bin.hip", "dm.hip", "grid.hip", "grow.hip", "segsdf.hip",
           "sizing.hip", "boundary.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def build(jobs: int = 5, verbose: bool = False) -> str:
    """Compile every source (always) and link libtrime.so."""
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs)
    _wait(procs)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    return LIB


def _wait(procs):
    errs = []
    while procs:
        src, p = procs.pop(0)
        out = p.communicate()[0].decode(errors="replace")
        if p.returncode != 0:
            errs.append("%s:\n%s" % (src, out))
        elif out.strip() and os.environ.get("TRIME_BUILD_VERBOSE"):
            print(out)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
