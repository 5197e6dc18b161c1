"""The C ABI from a plain C program (paper_1109_1264_amd/examples/fig1_dot.c,
built by the build step): no Python binding and no torch in that process,
only include/salt.h, libsalt.so and the HIP runtime. On the GPU its Fig. 1
result is bit for bit the oracle's and its dot is within the Dot2
tolerance and has the bits of the oracle's replay of the summation order."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import build as B
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads

T = S.token
FIG1 = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.LOAD, 2), T(S.SUB), T(S.ADD)]


def test_program_is_built_and_checks_its_arguments():
    """Built next to the library; without arguments it prints its usage and
    exits before touching the GPU."""
    assert os.path.exists(B.EXAMPLE), "run the build step first"
    p = subprocess.run([B.EXAMPLE], capture_output=True, text=True, timeout=60)
    assert p.returncode == 2 and "usage" in p.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 4099, 100003])
def test_fig1_and_dot_from_c(n, tmp_path):
    a, b, c = workloads.uniform(n, "f64", workloads.SEED_FIG1 + n, 3)
    paths = [tmp_path / x for x in ("a", "b", "c", "d", "dot")]
    for arr, p in zip((a, b, c), paths):
        np.ascontiguousarray(arr, dtype=np.float64).tofile(p)
    print("case n", n, flush=True)
    run = subprocess.run([B.EXAMPLE, str(n), *map(str, paths)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    d = np.fromfile(paths[3], dtype=np.float64)
    dot = float(np.fromfile(paths[4], dtype=np.float64)[0])
    want = oracle.eval_program(FIG1, [a, b, c], [], "f64")
    assert np.array_equal(d.view(np.uint64), want.view(np.uint64))
    ref, abs_sum = oracle.dot2(a, b)
    assert abs(dot - ref) <= oracle.TOL["f64"] * abs_sum
    assert dot == float(oracle.reduce_canonical("dot", a, b, "f64"))
