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
    "-I" + INCLUDE, "-I" + CSRC, "-I" + BUILD_DIR,
]

# Headers the run-time compiler (csrc/jit.hip) compiles kernels from: their
# text is embedded in the library, so a compiled tree, reduction pair or
# batched tree runs the same kernel template as the ahead-of-time ones.
JIT_HEADERS = [os.path.join(INCLUDE, "salt.h")] + [
    os.path.join(CSRC, h) for h in ("device.hpp", "expr.hpp", "eval_tree.hpp", "reduce_common.hpp",
                                    "reduce_tree.hpp", "batch.hpp", "batch_device.hpp")]
JIT_HEADERS_INC = os.path.join(BUILD_DIR, "jit_headers.inc")
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-I" + INCLUDE, "-I" + CSRC]
# A plain C program using the library through include/salt.h alone (no
# Python, no torch), built next to the library.
EXAMPLE_SRC = os.path.join(PKG, "examples", "fig1_dot.c")
EXAMPLE = os.path.join(PKG, "fig1_dot")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("build step failed: %s\n%s%s" % (" ".join(cmd), p.stdout, p.stderr))
    return p


def write_jit_headers(path: str = JIT_HEADERS_INC) -> None:
    """Write the embedded header table that csrc/jit.hip includes: the
    headers' names and their text as raw string literals."""
    delim = "SALT_HEADER_TEXT"
    names, texts = [], []
    for h in JIT_HEADERS:
        with open(h) as f:
            text = f.read()
        if ")" + delim in text:
            raise RuntimeError("%s contains the raw-string delimiter" % h)
        names.append('"%s"' % os.path.basename(h))
        texts.append('R"%s(%s)%s"' % (delim, text, delim))
    out = ("// Written by build.py: the headers the run-time compiler builds\n"
           "// reduction kernels from.\n"
           "static const int kJitHeaderCount = %d;\n"
           "static const char *const kJitHeaderNames[] = {%s};\n"
           "static const char *const kJitHeaderTexts[] = {\n%s};\n"
           % (len(names), ", ".join(names), ",\n".join(texts)))
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        f.write(out)
    os.replace(tmp, path)


def build(verbose: bool = False) -> str:
    """Compile every source and link ``libsalt.so``; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    write_jit_headers()
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
    build_example()
    return LIB


def build_example() -> str:
    """Compile examples/fig1_dot.c as C against the installed library and
    the HIP runtime; returns the program's path."""
    tmp = EXAMPLE + ".tmp%d" % os.getpid()
    _run(["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
          "-I" + INCLUDE, "-o", tmp, EXAMPLE_SRC, "-L" + PKG, "-lsalt", "-L" + os.path.join(ROCM, "lib"),
          "-lamdhip64", "-Wl,-rpath,$ORIGIN:" + os.path.join(ROCM, "lib")])
    os.replace(tmp, EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
