"""Fused tree -> reduction: dot(P, Q) and nrm2(P) in one pass must have the
same bits as evaluating P and Q into vectors (salt_eval) and reducing them
with salt_dot / salt_nrm2, and be within tolerance of the oracle's Dot2 of
the oracle-evaluated vectors."""
from __future__ import annotations

import random

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from tests.gpu_util import CODE, to_dev, empty

pytestmark = pytest.mark.gpu
T = S.token
DTYPES = ["f64", "f32", "bf16", "f16"]


@pytest.fixture(autouse=True)
def restore_jit_mode():
    yield
    S.salt_jit_set_mode(S.JIT_AUTO)


def composed(progs, dev, sc, dtype, n):
    import torch

    outs = []
    for p in progs:
        o = empty(n, dtype)
        S.salt_eval(p, dev, sc, o, n=n)
        outs.append(o)
    return outs


def rand_prog(rng, nops, nsc, leaves):
    def build(k):
        if k == 1:
            if nsc and rng.random() < 0.25:
                return [T(S.SCALAR, rng.randrange(nsc))]
            return [T(S.LOAD, rng.randrange(nops))]
        m = rng.randrange(1, k)
        return build(m) + build(k - m) + [T(rng.choice([S.ADD, S.SUB, S.MUL]))]
    return build(leaves)


@pytest.mark.parametrize("dtype", DTYPES)
def test_leaf_programs_equal_salt_dot(dtype):
    import torch

    Tt = S.salt_reduce_tile_elems(CODE[dtype])
    for n in (0, 1, 100, Tt - 3, Tt, 3 * Tt + 11, 300001):
        x, y = workloads.uniform(n, dtype, 60 + n % 97, 2)
        dx, dy = to_dev(x, dtype), to_dev(y, dtype)
        a = S.salt_dot_expr([T(S.LOAD, 0)], [T(S.LOAD, 1)], [dx, dy], [], n=n)
        b = S.salt_dot(dx, dy, n=n)
        c = S.salt_nrm2_expr([T(S.LOAD, 1)], [dx, dy], [], n=n)
        d = S.salt_nrm2(dy, n=n)
        torch.cuda.synchronize()
        assert a.item() == b.item(), (n, a.item(), b.item())
        assert c.item() == d.item(), (n, c.item(), d.item())


@pytest.mark.parametrize("dtype", DTYPES)
def test_fused_equals_composed_random_trees(dtype):
    import torch

    rng = random.Random(31337 + len(dtype))
    Tt = S.salt_reduce_tile_elems(CODE[dtype])
    for trial in range(24):
        nops, nsc = rng.randint(1, 6), rng.randint(0, 3)
        px = rand_prog(rng, nops, nsc, rng.randint(1, 6))
        py = rand_prog(rng, nops, nsc, rng.randint(1, 6))
        n = rng.choice([7, 5000, Tt + 1, 2 * Tt - 1, 100003])
        off = rng.choice([0, 0, 1])
        host = workloads.uniform(n, dtype, 900 + trial, nops)
        sc = [rng.uniform(-2, 2) for _ in range(nsc)]
        dev = [to_dev(h, dtype, offset=off) for h in host]
        print("trial", trial, dtype, n, off, px, py, flush=True)
        r = S.salt_dot_expr(px, py, dev, sc, n=n)
        q = S.salt_nrm2_expr(px, dev, sc, n=n)
        ex, ey = composed([px, py], dev, sc, dtype, n)
        r2 = S.salt_dot(ex, ey)
        q2 = S.salt_nrm2(ex)
        torch.cuda.synchronize()
        assert r.item() == r2.item(), (trial, r.item(), r2.item())
        assert q.item() == q2.item(), (trial, q.item(), q2.item())
        # and against the oracle's values
        vx = oracle.widen(oracle.eval_program(px, host, sc, dtype, n=n), dtype)
        vy = oracle.widen(oracle.eval_program(py, host, sc, dtype, n=n), dtype)
        ref, abs_sum = oracle.dot2(vx, vy)
        assert abs(r.item() - ref) <= oracle.TOL[dtype] * abs_sum + 1e-300


def test_deep_programs_swap_and_reject():
    import torch

    dtype = "f64"
    n = 40000
    host = workloads.uniform(n, dtype, 5, 8)
    dev = [to_dev(h, dtype) for h in host]
    deep = [T(S.LOAD, k) for k in range(8)] + [T(S.SUB)] * 7          # needs all 8 slots
    shallow = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL)]
    r = S.salt_dot_expr(deep, shallow, dev, [], n=n)
    ex, ey = composed([deep, shallow], dev, [], dtype, n)
    r2 = S.salt_dot(ex, ey)
    torch.cuda.synchronize()
    assert r.item() == r2.item()
    with pytest.raises(S.SaltError) as e:
        S.salt_dot_expr(deep, deep, dev, [], n=n)
    assert e.value.status == S.ERR_UNSUPPORTED


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_launch_shapes_do_not_change_bits(dtype):
    import torch

    n = 5 * S.salt_reduce_tile_elems(CODE[dtype]) + 333
    host = workloads.uniform(n, dtype, 4, 3)
    dev = [to_dev(h, dtype) for h in host]
    px = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD), T(S.LOAD, 2), T(S.MUL)]
    py = [T(S.LOAD, 2), T(S.SCALAR, 0), T(S.SUB)]
    ref = S.salt_dot_expr(px, py, dev, [0.5]).item()
    refn = S.salt_nrm2_expr(px, dev, [0.5]).item()
    for unroll in (2, 4, 8):
        for nt in (0, 1):
            for blocks in (0, 7, 256):
                cfg = (unroll, nt, blocks)
                assert S.salt_dot_expr(px, py, dev, [0.5], config=cfg).item() == ref, cfg
                assert S.salt_nrm2_expr(px, dev, [0.5], config=cfg).item() == refn, cfg


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_interpreter_unroll_shapes(dtype):
    """The interpreter's chunks-per-run knob does not change any bit."""
    import torch

    from tests.gpu_util import to_host_bits
    n = 123457
    host = workloads.uniform(n, dtype, 8, 3)
    dev = [to_dev(h, dtype) for h in host]
    prog = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD), T(S.LOAD, 2), T(S.MUL)]
    want = oracle.eval_program(prog, host, [], dtype)
    for unroll in (1, 2, 4, 8):
        for blocks in (0, 5, 300):
            out = empty(n, dtype)
            S.salt_eval(prog, dev, [], out, config=(unroll, 1, blocks))
            torch.cuda.synchronize()
            assert np.array_equal(to_host_bits(out, dtype), np.ascontiguousarray(want).view(to_host_bits(out, dtype).dtype)), (unroll, blocks)


# The reduction pairs with ahead-of-time kernels, each with an equivalent
# program pair that the catalogue does not match (an addition with its
# operands exchanged gives the same bits in IEEE arithmetic), so it runs on
# the interpreter.
L0, L1, L2, L3, S0 = T(S.LOAD, 0), T(S.LOAD, 1), T(S.LOAD, 2), T(S.LOAD, 3), T(S.SCALAR, 0)
PAIRS = {
    "dot_sum_diff": (([L0, L1, T(S.ADD)], [L0, L1, T(S.SUB)]), ([L1, L0, T(S.ADD)], [L0, L1, T(S.SUB)])),
    "nrm2_diff": (([L0, L1, T(S.SUB)], None), ([T(S.SCALAR, 1), L0, L1, T(S.SUB)] + [T(S.MUL)], None)),
    "nrm2_axpy": (([S0, L0, T(S.MUL), L1, T(S.ADD)], None), ([L1, S0, L0, T(S.MUL), T(S.ADD)], None)),
}


def run_pair(px, py, dev, sc, n, cfg=None):
    if py is None:
        return S.salt_nrm2_expr(px, dev, sc, n=n, config=cfg)
    return S.salt_dot_expr(px, py, dev, sc, n=n, config=cfg)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name", list(PAIRS))
def test_ahead_of_time_pairs(dtype, name):
    """Each catalogue pair routes to its ahead-of-time kernel and has the bits
    of (i) evaluating its trees with salt_eval and reducing the vectors, and
    (ii) the interpreter running an equivalent pair; and it is within the
    tolerance of the oracle's Dot2 of the oracle-evaluated vectors. Lengths
    cover the empty, single-tile, ragged and multi-tile cases, aligned and
    not."""
    import torch

    (px, py), (qx, qy) = PAIRS[name]
    # the equivalent pair runs on the interpreter (not on a compiled kernel)
    S.salt_jit_set_mode(S.JIT_OFF)
    assert S.salt_reduce_expr_route(px, py, 2, 2, CODE[dtype]) == list(PAIRS).index(name)
    assert S.salt_reduce_expr_route(qx, qy, 2, 2, CODE[dtype]) == -1
    # the interpreter variant of nrm2_diff multiplies by scalar 1 = 1.0 (exact)
    sc = [1.375, 1.0]
    Tt = S.salt_reduce_tile_elems(CODE[dtype])
    for n in (0, 1, 100, Tt - 3, Tt, Tt + 1, 3 * Tt + 11, 300001):
        for off in (0, 1):
            host = workloads.uniform(n, dtype, 70 + n % 89 + off, 2)
            dev = [to_dev(h, dtype, offset=off) for h in host]
            r = run_pair(px, py, dev, sc, n)
            r_int = run_pair(qx, qy, dev, sc, n)
            ex, ey = (composed([px, py], dev, sc, dtype, n) if py is not None
                      else composed([px], dev, sc, dtype, n) + [None])
            r_comp = S.salt_dot(ex, ey, n=n) if py is not None else S.salt_nrm2(ex, n=n)
            torch.cuda.synchronize()
            assert r.item() == r_comp.item(), (name, dtype, n, off, r.item(), r_comp.item())
            assert r.item() == r_int.item(), (name, dtype, n, off, r.item(), r_int.item())
            vx = oracle.widen(oracle.eval_program(px, host, sc, dtype, n=n), dtype)
            vy = vx if py is None else oracle.widen(oracle.eval_program(py, host, sc, dtype, n=n), dtype)
            ref, abs_sum = oracle.dot2(vx, vy)
            if py is None:
                assert abs(r.item() - np.sqrt(ref)) <= oracle.TOL[dtype] * np.sqrt(ref) + 1e-300
            else:
                assert abs(r.item() - ref) <= oracle.TOL[dtype] * abs_sum + 1e-300


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_ahead_of_time_pairs_launch_shapes_and_numbering(dtype):
    """Launch knobs do not change the bits of an ahead-of-time pair, and the
    pair is found under any operand numbering (operands 3 and 1 of four)."""
    import torch

    n = 5 * S.salt_reduce_tile_elems(CODE[dtype]) + 333
    host = workloads.uniform(n, dtype, 14, 4)
    dev = [to_dev(h, dtype) for h in host]
    px, py = [L3, L1, T(S.ADD)], [L3, L1, T(S.SUB)]
    assert S.salt_reduce_expr_route(px, py, 4, 0) == 0
    assert S.salt_reduce_expr_route(py, px, 4, 0) == 0          # programs exchanged
    ref = S.salt_dot_expr(px, py, dev, []).item()
    assert S.salt_dot_expr(py, px, dev, []).item() == ref
    ex, ey = composed([px, py], dev, [], dtype, n)
    assert S.salt_dot(ex, ey).item() == ref
    for unroll in (2, 4, 8, 16):
        for nt in (0, 1):
            for blocks in (0, 7, 256):
                cfg = (unroll, nt, blocks)
                assert S.salt_dot_expr(px, py, dev, [], config=cfg).item() == ref, cfg
