"""Parity of dot and nrm2 with the oracle's Dot2 values, within the stated
tolerances (FP64: 1e-13, FP32/16-bit storage: 1e-6, relative to
sum |x_i y_i| of the stored values), plus exact closed forms, bit-exact
determinism across repeats, launch shapes and alignment."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from tests.gpu_util import CODE, to_dev

pytestmark = pytest.mark.gpu

DTYPES = ["f64", "f32", "bf16", "f16"]


def tile(dtype):
    return S.salt_reduce_tile_elems(CODE[dtype])


def lengths(dtype):
    T = tile(dtype)
    return [0, 1, 5, 63, 64, 1000, T - 1, T, T + 1, 3 * T + 17, 1000003]


def gpu_dot(x, y, **kw):
    import torch

    r = S.salt_dot(x, y, **kw)
    torch.cuda.synchronize()
    return float(r.item())


def gpu_nrm2(x, **kw):
    import torch

    r = S.salt_nrm2(x, **kw)
    torch.cuda.synchronize()
    return float(r.item())


def check_dot(dtype, xh, yh, got):
    ref, abs_sum = oracle.dot2(oracle.widen(xh, dtype), oracle.widen(yh, dtype))
    tol = oracle.TOL[dtype] * abs_sum
    assert abs(got - ref) <= tol, (dtype, len(xh), got, ref, abs(got - ref) / max(abs_sum, 1e-300))


def check_nrm2(dtype, xh, got):
    w = oracle.widen(xh, dtype)
    ref = oracle.nrm2(w)
    # |r - ref| <= tol * ref: the sum's tolerance, halved by the root, plus
    # one rounding of the result
    tol = oracle.TOL[dtype] * ref
    assert abs(got - ref) <= tol, (dtype, len(xh), got, ref)


@pytest.mark.parametrize("dtype", DTYPES)
def test_dot_uniform(dtype):
    for k, n in enumerate(lengths(dtype)):
        x, y = workloads.uniform(n, dtype, 300 + k, 2)
        print("dot", dtype, n, flush=True)
        check_dot(dtype, x, y, gpu_dot(to_dev(x, dtype), to_dev(y, dtype)))


@pytest.mark.parametrize("dtype", DTYPES)
def test_nrm2_uniform(dtype):
    for k, n in enumerate(lengths(dtype)):
        (x,) = workloads.uniform(n, dtype, 400 + k, 1)
        print("nrm2", dtype, n, flush=True)
        got = gpu_nrm2(to_dev(x, dtype))
        if n == 0:
            assert got == 0.0
        else:
            check_nrm2(dtype, x, got)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_ill_conditioned(dtype):
    """Random signs, log10|x| ~ U[-4, 4]: large cancellation in the sum."""
    n = (1 << 20) + 333
    x64, y64 = workloads.ill_conditioned(n, workloads.SEED_PRECISION)
    x, y = workloads.store(x64, dtype), workloads.store(y64, dtype)
    dx, dy = to_dev(x, dtype), to_dev(y, dtype)
    check_dot(dtype, x, y, gpu_dot(dx, dy))
    check_nrm2(dtype, x, gpu_nrm2(dx))


def test_closed_forms():
    """a_i = i, b_i = 2i: dot = n(n-1)(2n-1)/3 exactly while every partial
    sum is an integer the accumulator holds exactly; ones: nrm2 = sqrt(n)."""
    for dtype, n in (("f64", 1 << 17), ("f64", 100001), ("f32", 256), ("f32", 200), ("bf16", 128), ("f16", 64)):
        i = np.arange(n, dtype=np.float64)
        x, y = workloads.store(i, dtype), workloads.store(2 * i, dtype)
        assert np.array_equal(oracle.widen(x, dtype), i) and np.array_equal(oracle.widen(y, dtype), 2 * i)
        got = gpu_dot(to_dev(x, dtype), to_dev(y, dtype))
        assert got == n * (n - 1) * (2 * n - 1) // 3, (dtype, n, got)
    for dtype in ("f64", "f32", "bf16", "f16"):
        for k in (0, 3, 8, 10):
            n = 4 ** k
            ones = workloads.store(np.ones(n), dtype)
            assert gpu_nrm2(to_dev(ones, dtype)) == 2.0 ** k


@pytest.mark.parametrize("dtype", DTYPES)
def test_deterministic_across_repeats_shapes_and_alignment(dtype):
    n = 5 * tile(dtype) + 12345
    x, y = workloads.uniform(n, dtype, 77, 2)
    dx, dy = to_dev(x, dtype), to_dev(y, dtype)
    ref = gpu_dot(dx, dy)
    check_dot(dtype, x, y, ref)
    for _ in range(20):
        assert gpu_dot(dx, dy) == ref
    for unroll in (2, 4, 8, 16):
        for nt in (0, 1):
            for blocks in (0, 1, 3, 64):
                assert gpu_dot(dx, dy, config=(unroll, nt, blocks)) == ref, (unroll, nt, blocks)
    # unaligned copies of the same values take the per-element path: same bits
    ux, uy = to_dev(x, dtype, offset=1), to_dev(y, dtype, offset=3)
    assert gpu_dot(ux, uy) == ref
    r2 = gpu_nrm2(dx)
    assert gpu_nrm2(to_dev(x, dtype, offset=5)) == r2
    assert gpu_nrm2(dx, config=(16, 1, 7)) == r2


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_precision_workload_full_size(dtype):
    """The precision workload at its full size: n = 2^26, random signs,
    log10|x| ~ U[-4, 4] (seed 3000), stored with round-to-nearest-even;
    dot and nrm2 within the tolerance of the oracle's Dot2 on the stored
    values."""
    n = 1 << 26
    x64, y64 = workloads.ill_conditioned(n, workloads.SEED_PRECISION)
    x, y = workloads.store(x64, dtype), workloads.store(y64, dtype)
    dx, dy = to_dev(x, dtype), to_dev(y, dtype)
    print("precision workload", dtype, n, flush=True)
    check_dot(dtype, x, y, gpu_dot(dx, dy))
    check_nrm2(dtype, x, gpu_nrm2(dx))


def test_bf16_products_outside_the_normal_range(orc):
    """The documented limits of the 16-bit accumulation: bfloat16 shares
    binary32's exponent range, so a product below 2^-126 is rounded as a
    binary32 subnormal (here (1 + 2^-7)^2 * 2^-140 keeps 9 significant bits:
    (1 + 2^-6) * 2^-140), and a product above the largest binary32 gives a
    non-finite result; binary16 products are exact."""
    import math

    import torch

    def bf16_bits(v):
        return np.array([orc.narrow(np.float32(v), "bf16")[0]] * 4, dtype=np.uint16)

    x = bf16_bits((1 + 2.0 ** -7) * 2.0 ** -70)           # exactly representable in bfloat16
    assert orc.widen(x, "bf16")[0] == (1 + 2.0 ** -7) * 2.0 ** -70
    dx = to_dev(x, "bf16")
    r = S.salt_dot(dx, dx)
    torch.cuda.synchronize()
    assert float(r.item()) == 4 * (1 + 2.0 ** -6) * 2.0 ** -140      # each product rounded
    exact, _ = orc.dot2(orc.widen(x, "bf16"), orc.widen(x, "bf16"))
    assert exact == 4 * (1 + 2.0 ** -6 + 2.0 ** -14) * 2.0 ** -140   # the oracle keeps every bit
    big = to_dev(bf16_bits(2.0 ** 70), "bf16")
    r = S.salt_dot(big, big)
    torch.cuda.synchronize()
    assert not math.isfinite(float(r.item()))
    # binary16: the product of two half-precision values is exact in binary32
    h = np.array([orc.narrow(np.float32(1 + 2.0 ** -10), "f16")[0]] * 4, dtype=np.uint16)
    r = S.salt_dot(to_dev(h, "f16"), to_dev(h, "f16"))
    torch.cuda.synchronize()
    assert float(r.item()) == 4 * (1 + 2.0 ** -10) ** 2
