"""Sharded reductions: a vector split at tile boundaries, pass 1 per shard
into one partial array (shard after shard), then one combine, gives the bits
of the one-call dot / nrm2 / asum -- the single-device part of a reduction
spread over several GPUs."""
from __future__ import annotations

import pytest

from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from tests.gpu_util import CODE, to_dev

pytestmark = pytest.mark.gpu

DTYPES = ["f64", "f32", "bf16", "f16"]


def whole(mode, x, y):
    if mode == S.MODE_DOT:
        return S.salt_dot(x, y)
    if mode == S.MODE_NRM2:
        return S.salt_nrm2(x)
    return S.salt_asum(x)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_shards_at_tile_boundaries_give_the_one_call_bits(dtype, mode):
    import torch

    T = S.salt_reduce_tile_elems(CODE[dtype])
    n = 5 * T + 77
    xh, yh = workloads.uniform(n, dtype, 4100 + mode, 2)
    x, y = to_dev(xh, dtype), to_dev(yh, dtype)
    want = float(whole(mode, x, y).item())
    for cuts in ([n], [2 * T, n], [T, 3 * T, 5 * T, n], [5 * T, n]):
        count = (n + T - 1) // T
        parts = torch.empty(count, dtype=torch.float64, device="cuda")
        lo, off = 0, 0
        for hi in cuts:
            m = hi - lo
            k = (m + T - 1) // T
            S.salt_reduce_partials(mode, x[lo:hi], y[lo:hi] if mode == S.MODE_DOT else None, n=m,
                                   partials=parts[off:off + k])
            lo, off = hi, off + k
        assert off == count
        got = float(S.salt_reduce_combine(mode, parts, CODE[dtype]).item())
        print("sharded", dtype, mode, cuts, flush=True)
        assert got == want, (dtype, mode, cuts, got, want)
    # no partials: zero
    empty = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert float(S.salt_reduce_combine(mode, empty, CODE[dtype], count=0).item()) == 0.0
