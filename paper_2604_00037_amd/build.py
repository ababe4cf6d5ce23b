"""Builds ``libaci.so`` (the HIP kernels and the C ABI) for gfx950 with hipcc.

Usage: ``python -m paper_2604_00037_amd.build`` or ``build_library()``.
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libaci.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 instructions are disabled for every kernel of the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


OBJ_DIR = os.path.join(ROOT, "_build")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build_library(verbose=False, extra_flags=()):
    """Compiles every source to an object in parallel, then links them into
    libaci.so (each translation unit keeps its own device code object)."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    jobs = []
    for src in sources():
        obj = os.path.join(OBJ_DIR, os.path.basename(src)[:-4] + ".o")
        jobs.append((obj, [hipcc, *flags, *extra_flags, "-I", os.path.join(ROOT, "include"), "-c", src,
                           "-o", obj]))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(workers) as ex:
        codes = list(ex.map(lambda j: _run(j[1], verbose), jobs))
    if any(codes):
        raise RuntimeError("hipcc failed compiling the sources of libaci.so")
    tmp = LIB + ".tmp"
    if _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *[j[0] for j in jobs], "-o", tmp], verbose):
        raise RuntimeError("hipcc failed linking libaci.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
