"""Builds libgmres_mi355x.so (HIP for gfx950) in-tree.

    python -m paper_1906_04051_amd.build [--release-only]

Each translation unit is compiled with hipcc in parallel into _build/, then
linked into the package directory.  Every HIP compile disables packed FP32
instructions (-packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgmres_mi355x.so")
SOURCES = ["krylov.hip", "adapt.hip", "setup.hip", "batched.hip", "block.hip", "api.cpp"]
ARCH = os.environ.get("GMRES_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


# roctx (marker ranges, GMRES_TRACE) from the ROCm installation.
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LINK = [f"-L{ROCM}/lib", f"-Wl,-rpath,{ROCM}/lib", "-lrocprofiler-sdk-roctx"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


# Bounds-checking variant (device checks of index ranges, see GM_DCHECK):
# same sources with -DGMRES_DEBUG, its own objects and library; load it with
# GMRES_LIB=<path of LIB_DEBUG>.
BUILD_DEBUG = os.path.join(HERE, "_build_debug")
LIB_DEBUG = os.path.join(HERE, "libgmres_mi355x_debug.so")


def _compile(job) -> str:
    src, debug = job
    obj = os.path.join(BUILD_DEBUG if debug else BUILD, os.path.splitext(src)[0] + ".o")
    extra = ["-DGMRES_DEBUG"] if debug else []
    cmd = [_hipcc(), *COMMON, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, *LINK]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, lib)


def build(verbose: bool = False, debug: bool = True) -> str:
    """Builds the release library and (debug=True) the bounds-checking one;
    the translation units compile in parallel."""
    variants = [False, True] if debug else [False]
    os.makedirs(BUILD, exist_ok=True)
    if debug:
        os.makedirs(BUILD_DEBUG, exist_ok=True)
    jobs = [(src, v) for v in variants for src in SOURCES]
    # The largest unit first, so it overlaps the others.
    jobs.sort(key=lambda j: j[0] != "krylov.hip")
    with cf.ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1, 8)) as ex:
        objs = dict(zip(jobs, ex.map(_compile, jobs)))
    _link([objs[(src, False)] for src in SOURCES], LIB)
    if verbose:
        print("built", LIB)
    if debug:
        _link([objs[(src, True)] for src in SOURCES], LIB_DEBUG)
        if verbose:
            print("built", LIB_DEBUG)
    return LIB


if __name__ == "__main__":
    build(verbose=True, debug="--release-only" not in sys.argv)
    sys.exit(0)
