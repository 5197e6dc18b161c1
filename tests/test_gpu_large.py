"""Sizes past 2^31 elements (64-bit indexing everywhere): binary16 vectors of
2^31 + 777 elements (4.3 GB each) on the device.

Element-wise results are checked on sampled indices (the boundary at 2^31,
the last tile, random positions) against the oracle evaluated on those
elements; reductions and iamax against closed forms that hold at any size."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from tests.gpu_util import to_host_bits

pytestmark = pytest.mark.gpu

N = (1 << 31) + 777
FIG1 = [S.token(S.LOAD, 0), S.token(S.LOAD, 1), S.token(S.LOAD, 2), S.token(S.SUB), S.token(S.ADD)]


def sample_indices(n, seed=5):
    rng = np.random.default_rng(seed)
    fixed = [0, 1, (1 << 31) - 2, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, n - 2, n - 1]
    return np.unique(np.concatenate([fixed, rng.integers(0, n, 4000)])).astype(np.int64)


def test_fig1_f16_past_2_31_sampled():
    import torch

    g = torch.Generator(device="cuda")
    g.manual_seed(1109)
    ops = [(torch.rand(N, device="cuda", generator=g, dtype=torch.float32) * 2 - 1).to(torch.float16)
           for _ in range(3)]
    out = torch.empty(N, dtype=torch.float16, device="cuda")
    print("fig1 f16 n =", N, flush=True)
    S.salt_eval(FIG1, ops, [], out)
    torch.cuda.synchronize()
    idx = sample_indices(N)
    ti = torch.from_numpy(idx).cuda()
    host_ops = [to_host_bits(o[ti], "f16") for o in ops]
    got = to_host_bits(out[ti], "f16")
    want = oracle.eval_program(FIG1, host_ops, [], "f16")
    assert np.array_equal(got, want), np.nonzero(got != want)[0][:5]
    del ops, out
    torch.cuda.empty_cache()


def test_reductions_and_iamax_past_2_31():
    import torch

    ones = torch.ones(N, dtype=torch.float16, device="cuda")
    print("dot / asum / nrm2 of ones, n =", N, flush=True)
    want = float(np.float32(N))  # the exact sum N, rounded once to binary32
    assert float(S.salt_dot(ones, ones).item()) == want
    assert float(S.salt_asum(ones).item()) == want
    assert float(S.salt_nrm2(ones).item()) == float(np.float32(np.sqrt(float(N))))
    # iamax: a planted maximum beyond 2^31, then an equal one early
    x = torch.zeros(N, dtype=torch.float16, device="cuda")
    far = (1 << 31) + 100
    x[far] = 5.0
    print("iamax n =", N, flush=True)
    assert int(S.salt_iamax(x).item()) == far
    x[7] = -5.0
    assert int(S.salt_iamax(x).item()) == 7
    # strided: the even positions only (element 7 is not one of them)
    m = (N + 1) // 2
    assert int(S.salt_iamax(x, m, 2).item()) == far // 2
    del ones, x
    torch.cuda.empty_cache()
