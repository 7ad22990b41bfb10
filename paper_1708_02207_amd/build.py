"""Compile the HDD HIP library (libhdd.so, in-tree) for gfx950 with hipcc.

Every source is compiled to its own object in parallel (the kernels of one
file never call another file's device code), then the objects are linked."""
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
LIB = os.path.join(PKG, "libhdd.so")
SOURCES = ["plan.cpp", "api.hip", "kernels_build.hip", "kernels_block.hip", "kernels_solve.hip", "kernels_func.hip",
           "kernels_lowrank.hip", "serve.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMPILE_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay disabled in every device code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
# roctx ranges around the host-side phases (csrc/trace.hpp)
LINK_FLAGS = ["-shared", "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def _run(cmd):
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Always recompiles (the build check must compile every time)."""
    jobs = jobs or min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    tmpdir = tempfile.mkdtemp(prefix="hdd_build_")
    try:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[HIPCC, *COMPILE_FLAGS, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(_run, cmds))
        for s, res in zip(SOURCES, results):
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed compiling {s}")
            if verbose:
                sys.stderr.write(res.stderr)
        tmp = LIB + ".tmp"
        res = _run([HIPCC, "--offload-arch=gfx950", *objs, *LINK_FLAGS, "-o", tmp])
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libhdd.so")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
