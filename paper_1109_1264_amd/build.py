"""Build ``libsalt.so`` (the HIP kernels and the C ABI) for gfx950, in tree.

    python -m paper_1109_1264_amd.build

Every HIP translation unit is compiled with contraction off (each add, sub
and mul stays one IEEE operation, as the element-wise results must be
bit-exact) and with packed binary32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsalt.so")

HIP_SOURCES = ["batch_f64.hip", "batch_f32.hip", "batch_bf16.hip", "batch_f16.hip",
               "reduce_f64.hip", "reduce_f32.hip", "reduce_bf16.hip", "reduce_f16.hip",
               "eval.hip", "reduce.hip", "batch.hip", "blas1.hip", "server.hip", "stream_ref.hip", "jit.hip", "api.hip"]
CXX_SOURCES = ["program.cpp"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
    "-I" + INCLUDE, "-I" + CSRC,
]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-I" + INCLUDE, "-I" + CSRC]


def _hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build step failed: %s\n%s%s" % (" ".join(cmd), p.stdout, p.stderr))
    return p


def build(verbose: bool = False) -> str:
    """Compile every source and link ``libsalt.so``; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD_DIR, src + ".o")
        jobs.append(([_hipcc(), *HIPCC_FLAGS, "-c", path, "-o", obj], obj))
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        jobs.append((["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    workers = min(len(jobs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(workers) as ex:
        for p in ex.map(lambda j: _run(j[0]), jobs):
            if verbose and p.stderr:
                sys.stderr.write(p.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp,
          *[o for _, o in jobs], "-ldl", "-lhiprtc"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
