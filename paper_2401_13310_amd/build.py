"""Builds the gfx950 shared library ``libhist.so`` of this package with hipcc.

The library is the product: every kernel and the C ABI of
``include/hist.h``.  It is compiled ahead of time for gfx950 only (no JIT,
no other targets), with packed-FP32 instructions disabled.  Each HIP source
is its own translation unit, compiled in parallel, then linked.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhist.so")
ARCH = "gfx950"

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def compile_command(src: str, obj: str) -> list:
    return ["hipcc"] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]


def link_command(objs: list, out: str) -> list:
    return ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out] + objs


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r.returncode, r.stdout + r.stderr


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every HIP source and links ``libhist.so`` (always recompiles)."""
    jobs = jobs or max(1, min(len(sources()), os.cpu_count() or 1, 16))
    tmpdir = tempfile.mkdtemp(prefix="histbuild_")
    try:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in sources()]
        cmds = [compile_command(s, o) for s, o in zip(sources(), objs)]
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        for cmd, (rc, out) in zip(cmds, results):
            if verbose:
                print(" ".join(cmd), flush=True)
            if rc != 0:
                sys.stderr.write(out)
                raise RuntimeError("hipcc failed compiling %s" % cmd[-3])
        tmp = LIB + ".tmp%d" % os.getpid()
        rc, out = _run(link_command(objs, tmp))
        if rc != 0:
            sys.stderr.write(out)
            raise RuntimeError("hipcc failed linking libhist.so")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
