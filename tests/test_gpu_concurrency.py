"""Calls from several host threads at once, each on its own stream: the
library's shared host state (the tuning table, the cache of run-time
compiled kernels, the per-thread error text) is used concurrently, and the
kernels of different streams overlap on the device. Every result must have
the bits of the same calls made one after another on one stream."""
from __future__ import annotations

import threading

import numpy as np
import pytest

from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from tests.gpu_util import to_dev, to_host_bits

pytestmark = pytest.mark.gpu
T = S.token

FIG1 = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.LOAD, 2), T(S.SUB), T(S.ADD)]
# outside the catalogue: interpreted at first, compiled at run time on its
# second large call (automatic mode), with the same bits either way
OTHER = [T(S.LOAD, 2), T(S.LOAD, 0), T(S.SUB), T(S.LOAD, 1), T(S.MUL), T(S.SCALAR, 0), T(S.ADD)]
PAIR_X = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 2), T(S.ADD)]
PAIR_Y = [T(S.LOAD, 1), T(S.SCALAR, 0), T(S.MUL)]


def work(dev, out, res, dtype, n):
    """The sequence each thread runs: element-wise calls (catalogue tree,
    a tree outside the catalogue three times), a dot, a norm and a fused
    expression dot; returns the device results."""
    S.salt_eval(FIG1, dev, [], out[0])
    for k in range(3):
        S.salt_eval(OTHER, dev, [0.375 + k], out[1 + k])
    r = [S.salt_dot(dev[0], dev[1], result=res[0]),
         S.salt_nrm2(dev[2], result=res[1]),
         S.salt_dot_expr(PAIR_X, PAIR_Y, dev, [1.5], result=res[2])]
    return r


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_threads_on_their_own_streams_match_serial_calls(dtype):
    import torch

    S.salt_jit_set_mode(S.JIT_AUTO)
    n = (1 << 17) + 77
    threads = 4
    tdt = torch.float64 if dtype == "f64" else torch.bfloat16
    rdt = torch.float64 if dtype == "f64" else torch.float32
    sets = []
    for t in range(threads):
        host = workloads.uniform(n, dtype, 8800 + t, 3)
        dev = [to_dev(h, dtype) for h in host]
        sets.append({
            "dev": dev,
            "out": [torch.empty(n, dtype=tdt, device="cuda") for _ in range(4)],
            "res": [torch.empty(1, dtype=rdt, device="cuda") for _ in range(3)],
            "ref_out": [torch.empty(n, dtype=tdt, device="cuda") for _ in range(4)],
            "ref_res": [torch.empty(1, dtype=rdt, device="cuda") for _ in range(3)],
        })
    torch.cuda.synchronize()
    errors = []
    start = threading.Barrier(threads)

    def run(s):
        try:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                start.wait(timeout=120)
                for _ in range(3):          # repeated, so calls of different threads interleave
                    work(s["dev"], s["out"], s["res"], dtype, n)
            stream.synchronize()
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    pool = [threading.Thread(target=run, args=(s,)) for s in sets]
    for th in pool:
        th.start()
    for th in pool:
        th.join()
    torch.cuda.synchronize()
    assert not errors, errors
    # the threads' repeated large calls compiled both trees outside the catalogue
    code = S.F64 if dtype == "f64" else S.BF16
    assert S.salt_eval_route(OTHER, 3, 1, code) == S.ROUTE_COMPILED
    assert S.salt_reduce_expr_route(PAIR_X, PAIR_Y, 3, 1, code) == S.ROUTE_COMPILED
    # the same calls one after another on the default stream (the threads
    # went first, so they also raced to compile the trees outside the
    # catalogue, while the others ran those trees interpreted)
    for s in sets:
        work(s["dev"], s["ref_out"], s["ref_res"], dtype, n)
    torch.cuda.synchronize()
    for t, s in enumerate(sets):
        for k in range(4):
            got, want = to_host_bits(s["out"][k], dtype), to_host_bits(s["ref_out"][k], dtype)
            assert np.array_equal(got, want), (t, k)
        for k in range(3):
            assert s["res"][k].item() == s["ref_res"][k].item(), (t, k, s["res"][k].item(), s["ref_res"][k].item())
