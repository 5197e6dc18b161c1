"""Reductions bit for bit against the oracle's replay of the library's
summation order (oracle.reduce_canonical): dot, nrm2 and asum in every
storage type, at lengths from 0 to more than 1024 tiles (so the final
combine's lanes take several partials), aligned and not; the hand-worked
order cases of the oracle's pins run through the device; and the paths
documented to give the same bits -- batched dots, strided reductions, and
the fused expression reductions -- against the same replay. Beside every
replay comparison sits the paper-anchored one: the result within the stated
tolerance of the oracle's Dot2 value (the replay follows the library's own
documented order, so its bits alone only show that the kernels implement
that order)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from paper_1109_1264_amd.batch import Batch
from tests.gpu_util import CODE, to_dev

pytestmark = pytest.mark.gpu

DTYPES = ["f64", "f32", "bf16", "f16"]
Tk = S.token


def bits(v) -> int:
    return int(np.float64(v).view(np.uint64))


def result(t) -> float:
    import torch

    torch.cuda.synchronize()
    return float(t.item())


def tile(dtype):
    return S.salt_reduce_tile_elems(CODE[dtype])


def within_dot2(got, mode, x, y, dtype):
    """The paper-anchored check beside the replay's bits: |got - Dot2| within
    the stated tolerance of sum |x_i y_i| (dot, asum) or of the norm."""
    wx = oracle.widen(x, dtype)
    if mode == "nrm2":
        ref = oracle.nrm2(wx)
        return abs(got - ref) <= oracle.TOL[dtype] * ref + 1e-300
    if mode == "asum":
        wx = np.abs(wx)
        wy = np.ones(len(wx))
    else:
        wy = oracle.widen(y, dtype)
    ref, abs_sum = oracle.dot2(wx, wy)
    return abs(got - ref) <= oracle.TOL[dtype] * abs_sum + 1e-300


def run(mode, xd, yd, n):
    if mode == "dot":
        return result(S.salt_dot(xd, yd, n=n))
    if mode == "nrm2":
        return result(S.salt_nrm2(xd, n=n))
    return result(S.salt_asum(xd, n, 1))


@pytest.mark.parametrize("dtype", DTYPES)
def test_contiguous_bits(dtype):
    T = tile(dtype)
    cases = [(0, 0), (1, 0), (5, 1), (63, 0), (1000, 1), (T - 1, 0), (T, 0), (T + 1, 1), (3 * T + 17, 0),
             (3 * T + 17, 1), (1000003, 0), (1030 * T + 77, 0)]
    for k, (n, off) in enumerate(cases):
        x, y = workloads.uniform(n, dtype, 8100 + k, 2)
        xd, yd = to_dev(x, dtype, offset=off), to_dev(y, dtype, offset=off)
        print("canonical", dtype, n, "offset", off, flush=True)
        for mode in ("dot", "nrm2", "asum"):
            got = run(mode, xd, yd, n)
            want = oracle.reduce_canonical(mode, x, y if mode == "dot" else None, dtype)
            assert bits(got) == bits(want), (dtype, mode, n, off, got, float(want))
        del xd, yd


def test_hand_worked_order_cases():
    """The oracle pins' order-dependent inputs (binary64): the device gives
    the hand-derived values (2^53 + 2 where a sequential sum gives 2^53)."""
    big = 2.0 ** 53
    T = tile("f64")
    cases = []
    x = np.zeros(T)
    x[0], x[1], x[512] = 2.0 ** 60, 1.0, -(2.0 ** 60)
    cases.append((x, 1.0))
    for idx, n in (((0, 4, 6), T), ((0, 256, 384), T), ((0, 2 * T, 3 * T), 4 * T), ((0, 128 * T, 192 * T), 193 * T)):
        x = np.zeros(n)
        x[idx[0]], x[idx[1]], x[idx[2]] = big, 1.0, 1.0
        cases.append((x, big + 2))
    for x, want in cases:
        got = result(S.salt_dot(to_dev(x, "f64"), to_dev(np.ones(len(x)), "f64")))
        assert got == want, (len(x), got, want)
        assert float(oracle.reduce_canonical("dot", x, np.ones(len(x)), "f64")) == want


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_batched_dots_bits(dtype):
    import torch

    T = tile(dtype)
    lengths = [1, 7, 63, T - 1, T, T + 1, 2 * T + 5] + [
        int(v) for v in workloads.batch_lengths(40, seed=9, median=2048, hi=1 << 17)]
    ops = [Tk(S.SCALAR, 0), Tk(S.LOAD, 0), Tk(S.MUL), Tk(S.LOAD, 1), Tk(S.LOAD, 2), Tk(S.SUB), Tk(S.ADD)]
    items, host = [], []
    for i, n in enumerate(lengths):
        a, b, c = workloads.uniform(n, dtype, 8300 + i, 3)
        off = i % 3 == 2
        dev = [to_dev(v, dtype, offset=int(off)) for v in (a, b, c)]
        r = torch.empty(1, dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
        items.append({"n": n, "operands": dev, "scalars": [1.5], "out": None, "dot_out": r})
        host.append((a, b))
    bt = Batch(ops, items, CODE[dtype])
    bt.launch()
    torch.cuda.synchronize()
    for it, (a, b) in zip(items, host):
        want = oracle.reduce_canonical("dot", a, b, dtype)
        got = float(it["dot_out"].item())
        assert bits(got) == bits(want), (dtype, it["n"])
        assert within_dot2(got, "dot", a, b, dtype), (dtype, it["n"])
    bt.close()


@pytest.mark.parametrize("dtype", DTYPES)
def test_strided_bits(dtype):
    T = tile(dtype)
    for k, (n, ix, iy) in enumerate([(5, 2, -3), (T + 1, 3, 1), (3 * T + 17, -2, 2), (200003, 1, -1)]):
        x = workloads.uniform(oracle.blas_span(n, ix), dtype, 8500 + k, 1)[0]
        y = workloads.uniform(oracle.blas_span(n, iy), dtype, 8600 + k, 1)[0]
        gx, gy = oracle.gather(n, x, ix), oracle.gather(n, y, iy)
        xd, yd = to_dev(x, dtype), to_dev(y, dtype)
        got = result(S.salt_dot_strided(xd, yd, n, ix, iy))
        assert bits(got) == bits(oracle.reduce_canonical("dot", gx, gy, dtype)), (dtype, n, ix, iy)
        assert within_dot2(got, "dot", gx, gy, dtype), (dtype, n, ix, iy)
        inc = abs(ix)
        got = result(S.salt_nrm2_strided(xd, n, inc))
        gi = oracle.gather(n, x, inc)
        assert bits(got) == bits(oracle.reduce_canonical("nrm2", gi, None, dtype)), (dtype, n, inc)
        assert within_dot2(got, "nrm2", gi, None, dtype), (dtype, n, inc)
        got = result(S.salt_asum(xd, n, inc))
        assert bits(got) == bits(oracle.reduce_canonical("asum", gi, None, dtype)), (dtype, n, inc)
        assert within_dot2(got, "asum", gi, None, dtype), (dtype, n, inc)


@pytest.mark.parametrize("dtype", DTYPES)
def test_fused_expression_reductions_bits(dtype):
    """dot(a + b, a - b) and nrm2(a*b - c): the replay over the oracle's
    evaluated (stored) vectors."""
    P = [Tk(S.LOAD, 0), Tk(S.LOAD, 1), Tk(S.ADD)]
    Q = [Tk(S.LOAD, 0), Tk(S.LOAD, 1), Tk(S.SUB)]
    R = [Tk(S.LOAD, 0), Tk(S.LOAD, 1), Tk(S.MUL), Tk(S.LOAD, 2), Tk(S.SUB)]
    T = tile(dtype)
    for k, n in enumerate([1, 1000, T - 1, 3 * T + 17]):
        a, b, c = workloads.uniform(n, dtype, 8700 + k, 3)
        dev = [to_dev(v, dtype) for v in (a, b, c)]
        px = oracle.eval_program(P, [a, b], [], dtype)
        qy = oracle.eval_program(Q, [a, b], [], dtype)
        got = result(S.salt_dot_expr(P, Q, dev[:2], [], n=n))
        assert bits(got) == bits(oracle.reduce_canonical("dot", px, qy, dtype)), (dtype, n)
        assert within_dot2(got, "dot", px, qy, dtype), (dtype, n)
        rz = oracle.eval_program(R, [a, b, c], [], dtype)
        got = result(S.salt_nrm2_expr(R, dev, [], n=n))
        assert bits(got) == bits(oracle.reduce_canonical("nrm2", rz, None, dtype)), (dtype, n)
        assert within_dot2(got, "nrm2", rz, None, dtype), (dtype, n)
