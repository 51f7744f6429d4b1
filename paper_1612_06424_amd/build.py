"""Build libdd.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1612_06424_amd.build

Every HIP source is compiled for gfx950 only, with packed-FP32 instructions
disabled (-Xclang -target-feature -Xclang -packed-fp32-ops), each in its own
hipcc process (several at once), then linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdd.so")
SOURCES = ["abi.hip", "dirac.hip", "blas.hip", "krylov.hip", "solver.hip", "evenodd.hip", "batched.hip", "tune.hip",
           "projection.hip", "disconnected.hip", "nucleon.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    tmpdir = tempfile.mkdtemp(prefix="dd_build_")
    try:
        def compile_one(src):
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc, *FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
            return obj

        # the heaviest sources first, so that they start at once
        order = sorted(SOURCES, key=lambda s: -os.path.getsize(os.path.join(CSRC, s)))
        with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
            objs = dict(zip(order, pool.map(compile_one, order)))
        tmp = LIB + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-fPIC", "-shared", *[objs[s] for s in SOURCES], "-o", tmp,
               "-Wl,-rpath,/opt/rocm/lib"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
