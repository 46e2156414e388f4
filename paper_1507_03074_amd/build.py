"""Builds libht.so (the HIP kernels and the C ABI) in-tree for gfx950 with hipcc.

Each translation unit compiles to its own object, in parallel; the fill kernel's row counts are
separate objects of one source (ht_fill_rows.hip with -DHT_FILL_ROWS=n). The objects are then
linked into one shared library.

Usage: python -m paper_1507_03074_amd.build   (or __graft_entry__.build())
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libht.so")

FILL_ROWS = (1, 2, 4, 8, 16, 32, 64)
# (source, extra defines) of every object
UNITS = ([("ht_kernels.hip", []), ("ht_api.cpp", []), ("ht_serve.cpp", []), ("ht_roofline.hip", []),
          ("ht_noalloc.hip", [])] +
         [("ht_fill_rows.hip", ["-DHT_FILL_ROWS=%d" % r]) for r in FILL_ROWS])

# -ffp-contract=off: the bin rule is one rounding per operation, never a fused multiply-add.
# -packed-fp32-ops: keep the compiler from emitting packed FP32 arithmetic.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-pthread",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16, len(UNITS)))


def build(verbose: bool = False) -> str:
    tmpdir = tempfile.mkdtemp(prefix="htbuild")
    try:
        def compile_one(i):
            src, defs = UNITS[i]
            obj = os.path.join(tmpdir, "%02d_%s.o" % (i, os.path.splitext(src)[0]))
            cmd = [hipcc(), *HIPCC_FLAGS, *defs, "-I", INCLUDE, "-I", CSRC, "-c",
                   os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
            return obj

        with ThreadPoolExecutor(_jobs()) as pool:
            objs = list(pool.map(compile_one, range(len(UNITS))))
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


def stale() -> bool:
    """Whether libht.so is missing or older than any of its sources and headers."""
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + \
        [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
    return any(os.path.getmtime(d) > t for d in deps)


def ensure_built() -> str:
    """Builds libht.so when it is missing or stale; returns its path."""
    if stale():
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
