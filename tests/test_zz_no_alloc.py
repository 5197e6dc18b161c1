"""salt_dot_noalloc (the dot that takes no workspace) against salt_dot, the
entry point it is a variant of: the same bits on two calls in a row, the
second with a smaller input (the shared partials buffer keeps the first
call's values), in every storage type, plus the Dot2 tolerance of the
oracle, the largest length the built-in buffer allows, and the size
limit."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads

pytestmark = pytest.mark.gpu

TDT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16"}
CODE = {"f64": S.F64, "f32": S.F32, "bf16": S.BF16, "f16": S.F16}
TOL = {"f64": 1e-13, "f32": 1e-6, "bf16": 1e-6, "f16": 1e-6}


def dev_operands(n, dt, seed):
    return workloads.uniform_device(n, dt, seed, 2)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16", "f16"])
def test_two_calls_in_a_row_match_salt_dot(dt, orc):
    import torch

    sizes = (3 * S.salt_reduce_tile_elems(CODE[dt]) * 37 + 1234, 40000 + 7)   # second call smaller
    for k, n in enumerate(sizes):
        x, y = dev_operands(n, dt, 900 + k)
        r_ref = S.salt_dot(x, y)
        r_new = S.salt_dot_noalloc(x, y)
        torch.cuda.synchronize()
        assert torch.equal(r_new.view(torch.uint8), r_ref.view(torch.uint8)), (dt, n)
        # and within the oracle's tolerance of the Dot2 value of the stored values
        bits = lambda t: (t.view(torch.int16).cpu().numpy().view(np.uint16) if dt in ("bf16", "f16")
                          else t.cpu().numpy())
        wx, wy = orc.widen(bits(x), dt), orc.widen(bits(y), dt)
        ref, abs_sum = orc.dot2(wx, wy)
        assert abs(float(r_new.item()) - ref) <= TOL[dt] * abs_sum


def test_empty_and_single_tile():
    import torch

    x, y = dev_operands(1000, "f64", 5)
    r = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    S.salt_dot_noalloc(x, y, n=0, result=r)
    torch.cuda.synchronize()
    assert r.item() == 0.0
    r1, r2 = S.salt_dot_noalloc(x, y), S.salt_dot(x, y)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)


def test_largest_length_and_the_limit():
    """n = 2^30 binary64 elements fills the buffer's 2^17 partials exactly;
    one element more is refused before anything is enqueued."""
    import torch

    n = 1 << 30
    assert S.salt_reduce_workspace_bytes(n, S.F64) == 131072 * 8
    x = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    y = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    y[1::2] = -1.0
    r1 = S.salt_dot_noalloc(x, y)
    r2 = S.salt_dot(x, y)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)
    assert r1.item() == n / 4            # n/2 products of +1 and n/2 of -0.5, all exact
    L = S.lib()
    r = torch.empty(1, dtype=torch.float64, device="cuda")
    st = L.salt_dot_noalloc(n + 1, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                            ctypes.c_void_p(r.data_ptr()), S.F64, None)
    assert st == S.ERR_UNSUPPORTED
    del x, y
    torch.cuda.empty_cache()


def test_ordered_calls_on_one_stream_reuse_the_buffer():
    """Several calls queued back to back on one stream, each a different
    length: every result equals salt_dot's."""
    import torch

    outs, refs = [], []
    for k, n in enumerate((1 << 22, 5 * 8192 + 3, 1 << 20, 100)):
        x, y = dev_operands(n, "f64", 950 + k)
        outs.append(S.salt_dot_noalloc(x, y))
        refs.append(S.salt_dot(x, y))
    torch.cuda.synchronize()
    for a, b in zip(outs, refs):
        assert torch.equal(a, b)
