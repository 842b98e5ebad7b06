"""Builds run_case: the library's kernels and host code compiled for the CPU
against the stand-in HIP runtime (hip/hip_runtime.h, emu.cpp), with
AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure).

The product sources are copied with two textual changes, each applied
exactly once:
- global loads and stores, and LDS pointers passed to functions, lose
  their address-space qualifier, which AddressSanitizer does not
  instrument;
- the polygons of the wavefront-per-point passes (one polygon per wavefront
  or per group of 8 lanes, which every lane of the group reads and writes
  with identical values in lockstep on the GPU) become per-lane arrays,
  since the emulation runs lanes one after another between barriers.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
# EMU_SRC: another copy of the package's sources and headers (a directory
# holding pkg/csrc and include), for trying changes before they are made
SRC_ROOT = os.environ.get("EMU_SRC")
CSRC = os.path.join(SRC_ROOT, "pkg", "csrc") if SRC_ROOT else os.path.join(ROOT, "paper_2309_13824_amd", "csrc")
INCLUDE = os.path.join(SRC_ROOT, "include") if SRC_ROOT else os.path.join(ROOT, "include")
OUT_NAME = "_build_alt" if SRC_ROOT else "_build"
OUT = os.path.join(HERE, OUT_NAME)
EXE = os.path.join(OUT, "run_case")
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")

EDITS = {
    "trime_dev.hpp": [("#define TRIME_GLOBAL __attribute__((address_space(1)))", "#define TRIME_GLOBAL"),
                      ("#define TRIME_LDS __attribute__((address_space(3)))", "#define TRIME_LDS")],
    "cells_k.hpp": [("auto &P = sh.P;", "VRec<double> P[VMAX][1];"),
                    ("auto &PC = sh.PC;", "VRec<double> PC[V][8];")],
}
SOURCES = ["abi.hip", "adapt.hip", "bin.hip", "cells.hip", "dm.hip", "grid.hip", "grow.hip", "segsdf.hip",
           "sizing.hip", "boundary.hip", "persist.hip"]
# TRIME_PERSIST_ENABLE: the persistent batch kernel, switched off in the
# device build, is built in here
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-ffp-contract=off", "-Wno-unused-result", "-DTRIME_PERSIST_ENABLE"]


def prepare():
    src = os.path.join(OUT, "pkg", "csrc")
    os.makedirs(src, exist_ok=True)
    os.makedirs(os.path.join(OUT, "include"), exist_ok=True)
    shutil.copy(os.path.join(INCLUDE, "trime.h"), os.path.join(OUT, "include", "trime.h"))
    for f in os.listdir(CSRC):
        if not f.endswith((".hip", ".hpp")):
            continue
        text = open(os.path.join(CSRC, f)).read()
        for old, new in EDITS.get(f, []):
            if text.count(old) != 1:
                raise RuntimeError("%s: expected one '%s', found %d" % (f, old, text.count(old)))
            text = text.replace(old, new)
        dst = os.path.join(src, f)
        if not os.path.exists(dst) or open(dst).read() != text:
            with open(dst, "w") as fh:
                fh.write(text)
    return src


def build(jobs=8):
    src = prepare()
    inc = ["-I", HERE, "-I", os.path.join(OUT, "include")]
    jobs_ = []
    objs = []
    units = [(os.path.join(src, s), ["-x", "c++"]) for s in SOURCES]
    units += [(os.path.join(HERE, "emu.cpp"), []), (os.path.join(HERE, "run_case.cpp"), [])]
    for path, lang in units:
        obj = os.path.join(OUT, os.path.basename(path) + ".o")
        objs.append(obj)
        if os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(path), _newest_header(src)):
            continue
        cmd = [CXX] + FLAGS + inc + lang + ["-c", path, "-o", obj]
        jobs_.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        if len(jobs_) >= jobs:
            _wait(jobs_)
    _wait(jobs_)
    r = subprocess.run([CXX] + FLAGS + objs + ["-o", EXE], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    if r.returncode:
        raise RuntimeError("link failed:\n" + r.stdout)
    return EXE


def _newest_header(src):
    t = os.path.getmtime(os.path.join(HERE, "hip", "hip_runtime.h"))
    for f in os.listdir(src):
        if f.endswith(".hpp"):
            t = max(t, os.path.getmtime(os.path.join(src, f)))
    return max(t, os.path.getmtime(os.path.join(OUT, "include", "trime.h")))


def _wait(jobs_):
    errs = []
    while jobs_:
        p = jobs_.pop(0)
        out = p.communicate()[0].decode(errors="replace")
        if p.returncode:
            errs.append(out)
    if errs:
        raise RuntimeError("compile failed:\n" + "\n".join(errs)[:20000])


if __name__ == "__main__":
    print(build())
    sys.exit(0)
