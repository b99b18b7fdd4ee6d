"""Build the gfx950 HIP library libgn.so in-tree with hipcc.

The library is the product: hand-written HIP kernels plus the C ABI of
include/gn.h.  It is compiled for gfx950 only, with packed-FP32 instruction
selection disabled and no fast-math (FP64 semantics: IEEE, denormals kept).
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libgn.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src: str, obj: str) -> subprocess.CompletedProcess:
    cmd = [HIPCC, *FLAGS, "-c", "-I", INCLUDE, "-I", CSRC, src, "-o", obj]
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source (one hipcc per file, in parallel) and link
    libgn.so.  Always recompiles.  Each translation unit launches only its own
    kernels, so the objects link without relocatable device code."""
    srcs = sources()
    objdir = tempfile.mkdtemp(prefix="gn_build_")
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, os.cpu_count() or 1), 16)
    if verbose:
        print("compiling %d sources with %d jobs" % (len(srcs), jobs), flush=True)
    try:
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(_compile, srcs, objs))
        bad = [(s, r) for s, r in zip(srcs, results) if r.returncode != 0]
        for s, r in bad:
            sys.stderr.write("%s:\n%s%s" % (s, r.stdout, r.stderr))
        if bad:
            raise RuntimeError("hipcc failed on %s" % ", ".join(os.path.basename(s) for s, _ in bad))
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libgn.so")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
