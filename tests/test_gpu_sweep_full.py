"""The BLAS-1 sweep at its largest size, n = 2^28, in binary64 and binary32,
with the tuned launch knobs (the configuration the benchmark times):
the 5-operand tree and axpy bit-exact on sampled elements (the boundary
tiles and 2^16 random positions) against the oracle evaluated on those
elements; dot and nrm2 within tolerance of the oracle over all elements."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads

pytestmark = pytest.mark.gpu

T = S.token
TREE5 = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 2), T(S.LOAD, 3), T(S.MUL), T(S.ADD), T(S.LOAD, 4),
         T(S.SUB)]
AXPY = [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL), T(S.LOAD, 1), T(S.ADD)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sweep_largest_size(dtype):
    import torch

    n = 1 << 28
    seed = workloads.sweep_seed(n)
    al = workloads.alpha(seed)
    a, b, c, e, f = workloads.uniform_device(n, dtype, seed, 5)
    d = torch.empty_like(a)
    y = f.clone()
    print("sweep largest size", dtype, flush=True)
    S.salt_eval(TREE5, [a, b, c, e, f], [], d)
    S.salt_axpy(al, a, y)
    r_dot = S.salt_dot(a, b)
    r_nrm = S.salt_nrm2(c)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(7))
    idx = np.unique(np.concatenate([rng.integers(0, n, 1 << 16), np.arange(4096), np.arange(n - 4096, n)]))
    ti = torch.from_numpy(idx).cuda()
    ops = [t.index_select(0, ti).cpu().numpy() for t in (a, b, c, e, f)]
    got = d.index_select(0, ti).cpu().numpy()
    want = oracle.eval_program(TREE5, ops, [], dtype)
    assert np.array_equal(got.view(np.uint8), want.view(np.uint8))
    got = y.index_select(0, ti).cpu().numpy()
    want = oracle.eval_program(AXPY, [ops[0], ops[4]], [al], dtype)
    assert np.array_equal(got.view(np.uint8), want.view(np.uint8))
    ah, bh = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
    ref, abs_sum = oracle.dot2(ah, bh)
    assert abs(float(r_dot.item()) - ref) <= oracle.TOL[dtype] * abs_sum
    del ah, bh
    ch = c.cpu().numpy().astype(np.float64)
    nref = oracle.nrm2(ch)
    assert abs(float(r_nrm.item()) - nref) <= oracle.TOL[dtype] * nref
    del a, b, c, e, f, d, y
    torch.cuda.empty_cache()
