"""Build the HIP library libcasimir_fdtd.so in-tree for gfx950.

    python -m paper_0906_5170_amd.build        (or __graft_entry__.build())

Every source under csrc/ is compiled by hipcc (one process per source, in
parallel) and linked into one shared library that exports the C ABI of
include/casimir_fdtd.h.  Each .hip file launches its own kernels through
host wrappers, so the translation units need no relocatable device code.
Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcasimir_fdtd.so")
ARCH = os.environ.get("CF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, name))
    return out


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmpdir = tempfile.mkdtemp(prefix="cf_build_")
    try:
        srcs = sources()
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]

        def compile_one(k):
            cmd = [hipcc, *HIPCC_FLAGS, "-c", srcs[k], "-o", objs[k]]
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
        with ThreadPoolExecutor(jobs) as pool:
            results = list(pool.map(compile_one, range(len(srcs))))
        failed = False
        for s, r in zip(srcs, results):
            # hipcc's host pass warns that it does not know the packed-FP32
            # feature; that line is expected and not repeated here
            err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
            if err.strip():
                print(err, file=sys.stderr, flush=True)
            if r.returncode != 0:
                print(f"compile failed: {s}", file=sys.stderr, flush=True)
                failed = True
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc")
        tmp = LIB + ".tmp"
        cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
