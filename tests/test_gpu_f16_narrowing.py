"""binary16 results are rounded twice, as the arithmetic says: each
operation to binary32, then the stored value to binary16. A multiply
followed by the narrowing must not become one mixed-precision fused
instruction that rounds the exact product to binary16 once (gfx950 has
such instructions, and the compiler forms them from that pattern). The
inputs here make the two roundings differ on thousands of elements (checked
on the host first), on every path that narrows: whole tiles, element-wise
tails and unaligned views, strided scal, the run-time compiled tree, the
batched kernels (ahead of time and compiled) and the reductions' store
rounding."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from paper_1109_1264_amd.batch import Batch
from tests.gpu_util import empty, first_mismatch, oracle_bits, to_dev, to_host_bits

T = S.token
ALPHA = 1.9255319833755493          # a binary32 value (the scalar is rounded to it)
SCALE = [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL)]                          # catalogue tree
ABA = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.SCALAR, 0), T(S.MUL)]   # (a*b)*alpha, compiled
N = (1 << 20) + 13


def inputs(k=1, seed=8800):
    return workloads.uniform(N, "f16", seed, k)


def sensitive(a_bits):
    """How many elements round differently once than twice (host)."""
    a = np.asarray(a_bits, dtype=np.uint16).view(np.float16).astype(np.float64)
    exact = a * float(np.float32(ALPHA))                     # exact in binary64
    return int(np.count_nonzero(exact.astype(np.float16) != exact.astype(np.float32).astype(np.float16)))


def eval_bits(prog, dev, sc, n, offset=0, cfg=None):
    import torch

    out = empty(n, "f16", offset=offset)
    S.salt_eval(prog, dev, sc, out, n=n, config=cfg)
    torch.cuda.synchronize()
    return to_host_bits(out, "f16")


def test_inputs_are_sensitive():
    """(host) The inputs make the two roundings differ on many elements."""
    (a,) = inputs()
    assert sensitive(a) > 1000


@pytest.mark.gpu
@pytest.mark.parametrize("offset", [0, 1])
def test_scale_tree(offset):
    (a,) = inputs()
    want = oracle_bits(oracle.eval_program(SCALE, [a], [ALPHA], "f16"), "f16")
    dev = [to_dev(a, "f16", offset=offset)]
    for cfg in (None, (1, 1, 0), (8, 0, 64)):
        got = eval_bits(SCALE, dev, [ALPHA], N, offset=offset, cfg=cfg)
        assert np.array_equal(got, want), (offset, cfg, first_mismatch(got, want))


@pytest.mark.gpu
@pytest.mark.parametrize("offset", [0, 1])
def test_compiled_tree(offset):
    a, b = inputs(2, seed=8810)
    b = np.full(N, np.float16(1.0).view(np.uint16), dtype=np.uint16)      # (a*1)*alpha: a*alpha
    want = oracle_bits(oracle.eval_program(ABA, [a, b], [ALPHA], "f16"), "f16")
    S.salt_jit_set_mode(S.JIT_EXPLICIT)
    try:
        S.salt_jit_compile(ABA, 2, 1, S.F16)
        assert S.salt_eval_route(ABA, 2, 1, S.F16) == S.ROUTE_COMPILED
        got = eval_bits(ABA, [to_dev(a, "f16", offset=offset), to_dev(b, "f16", offset=offset)], [ALPHA], N,
                        offset=offset)
        assert np.array_equal(got, want), first_mismatch(got, want)
        S.salt_jit_set_mode(S.JIT_OFF)                                 # and the interpreter
        got = eval_bits(ABA, [to_dev(a, "f16", offset=offset), to_dev(b, "f16", offset=offset)], [ALPHA], N,
                        offset=offset)
        assert np.array_equal(got, want), first_mismatch(got, want)
    finally:
        S.salt_jit_set_mode(S.JIT_AUTO)


@pytest.mark.gpu
def test_strided_scal():
    import torch

    (a,) = inputs(seed=8820)
    m = N // 2
    x = to_dev(a, "f16")
    S.salt_scal(ALPHA, x, m, 2)
    torch.cuda.synchronize()
    want = oracle_bits(oracle.scal(m, ALPHA, a, 2, "f16"), "f16")
    got = to_host_bits(x, "f16")
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.gpu
@pytest.mark.parametrize("prog", ["scale", "compiled"])
def test_batched(prog):
    import torch

    tree = SCALE if prog == "scale" else ABA
    lengths = [N, 4097, 1, 65536 + 3]
    items, want = [], []
    one = np.float16(1.0).view(np.uint16)
    for i, n in enumerate(lengths):
        (a,) = workloads.uniform(n, "f16", 8830 + i, 1)
        b = np.full(n, one, dtype=np.uint16)
        off = i % 2
        ops = [to_dev(a, "f16", offset=off)] + ([to_dev(b, "f16", offset=off)] if prog == "compiled" else [])
        items.append({"n": n, "operands": ops, "scalars": [ALPHA], "out": empty(n, "f16", offset=off),
                      "dot_out": None})
        host = [a] if prog == "scale" else [a, b]
        want.append(oracle_bits(oracle.eval_program(tree, host, [ALPHA], "f16"), "f16"))
    bt = Batch(tree, items, S.F16)
    bt.launch()
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        got = to_host_bits(it["out"], "f16")
        assert np.array_equal(got, want[i]), (i, first_mismatch(got, want[i]))
    bt.close()


@pytest.mark.gpu
@pytest.mark.parametrize("offset", [0, 1])
def test_reduction_store_rounding(offset):
    """nrm2(alpha*a) in one pass rounds alpha*a to binary16 as salt_eval
    would store it: the same bits as evaluating and then reducing."""
    import torch

    (a,) = inputs(seed=8840)
    dev = [to_dev(a, "f16", offset=offset)]
    S.salt_jit_set_mode(S.JIT_OFF)
    try:
        fused_int = S.salt_nrm2_expr(SCALE, dev, [ALPHA])
        S.salt_jit_set_mode(S.JIT_EXPLICIT)
        S.salt_jit_compile_reduce(SCALE, None, 1, 1, S.F16)
        fused_jit = S.salt_nrm2_expr(SCALE, dev, [ALPHA])
    finally:
        S.salt_jit_set_mode(S.JIT_AUTO)
    out = empty(N, "f16")
    S.salt_eval(SCALE, dev, [ALPHA], out)
    composed = S.salt_nrm2(out)
    torch.cuda.synchronize()
    assert fused_int.item() == composed.item() == fused_jit.item()
    v = oracle.widen(oracle.eval_program(SCALE, [a], [ALPHA], "f16"), "f16")
    ref, _ = oracle.dot2(v, v)
    assert abs(composed.item() - np.sqrt(ref)) <= oracle.TOL["f16"] * np.sqrt(ref)
