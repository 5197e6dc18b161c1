"""Trees outside the catalogue on their run-time compiled kernels: bit for
bit against the oracle and against the interpreter, in every element type,
at lengths spanning several tiles and ragged tails, aligned and not, in
place, under every launch shape; the automatic mode compiles a tree at its
second large call without changing a bit; a launch captured into a HIP
graph before the kernel is loaded runs interpreted and replays correctly.
The same for reduction pairs outside the reduction catalogue (dot and nrm2
of expressions): the compiled pass 1 gives the interpreter's bits, within
the tolerance of the oracle's Dot2 of the oracle-evaluated vectors."""
from __future__ import annotations

import random

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from tests.gpu_util import CODE, empty, to_dev, to_host_bits

pytestmark = pytest.mark.gpu
T = S.token
DTYPES = ["f64", "f32", "bf16", "f16"]


def rand_prog(rng, nops, nsc, leaves):
    def build(k):
        if k == 1:
            if nsc and rng.random() < 0.25:
                return [T(S.SCALAR, rng.randrange(nsc))]
            return [T(S.LOAD, rng.randrange(nops))]
        m = rng.randrange(1, k)
        return build(m) + build(k - m) + [T(rng.choice([S.ADD, S.SUB, S.MUL]))]
    return build(leaves)


@pytest.fixture(autouse=True)
def restore_mode():
    yield
    S.salt_jit_set_mode(S.JIT_AUTO)


def eval_bits(prog, dev, sc, dtype, n, cfg=None):
    import torch

    out = empty(n, dtype)
    S.salt_eval(prog, dev, sc, out, n=n, config=cfg)
    torch.cuda.synchronize()
    return to_host_bits(out, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_compiled_trees_against_oracle_and_interpreter(dtype):
    rng = random.Random(4242 + len(dtype))
    for trial in range(10):
        nops, nsc = rng.randint(1, 8), rng.randint(0, 3)
        prog = rand_prog(rng, nops, nsc, rng.randint(2, 8))
        S.salt_jit_set_mode(S.JIT_EXPLICIT)
        S.salt_jit_compile(prog, nops, nsc, CODE[dtype])
        if S.salt_eval_route(prog, nops, nsc, CODE[dtype]) >= 0:
            continue                                   # drew a catalogue tree
        assert S.salt_eval_route(prog, nops, nsc, CODE[dtype]) == S.ROUTE_COMPILED
        n = rng.choice([1, 777, 65536 + 13, 300007])
        off = rng.choice([0, 0, 1])
        host = workloads.uniform(n, dtype, 6100 + trial, nops)
        sc = [rng.uniform(-2, 2) for _ in range(nsc)]
        dev = [to_dev(h, dtype, offset=off) for h in host]
        print("jit trial", trial, dtype, n, off, prog, flush=True)
        got = eval_bits(prog, dev, sc, dtype, n)
        want = np.ascontiguousarray(oracle.eval_program(prog, host, sc, dtype)).view(got.dtype)
        assert np.array_equal(got, want), (trial, dtype, n, off)
        S.salt_jit_set_mode(S.JIT_OFF)
        assert np.array_equal(eval_bits(prog, dev, sc, dtype, n), got), (trial, "interpreter")


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_launch_shapes_and_in_place(dtype):
    import torch

    S.salt_jit_set_mode(S.JIT_EXPLICIT)
    prog = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD), T(S.LOAD, 2), T(S.MUL)]      # (a + b) * c
    S.salt_jit_compile(prog, 3, 0, CODE[dtype])
    assert S.salt_eval_route(prog, 3, 0, CODE[dtype]) == S.ROUTE_COMPILED
    n = 5 * 256 * 4 * 8 + 1234
    host = workloads.uniform(n, dtype, 6300, 3)
    dev = [to_dev(h, dtype) for h in host]
    want = np.ascontiguousarray(oracle.eval_program(prog, host, [], dtype))
    for unroll in (1, 2, 4, 8):
        for nt in (0, 1):
            for blocks in (0, 3, 1000):
                got = eval_bits(prog, dev, [], dtype, n, cfg=(unroll, nt, blocks))
                assert np.array_equal(got, want.view(got.dtype)), (unroll, nt, blocks)
    # in place: the output is operand 2
    S.salt_eval(prog, dev, [], dev[2])
    torch.cuda.synchronize()
    got = to_host_bits(dev[2], dtype)
    assert np.array_equal(got, want.view(got.dtype))


def test_automatic_mode_switches_without_changing_bits():
    S.salt_jit_set_mode(S.JIT_AUTO)
    # a tree no other test uses: (a - b) * (c - a) * alpha, binary32
    prog = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.SUB), T(S.LOAD, 2), T(S.LOAD, 0), T(S.SUB), T(S.MUL),
            T(S.SCALAR, 0), T(S.MUL)]
    n = 1 << 18
    host = workloads.uniform(n, "f32", 6400, 3)
    dev = [to_dev(h, "f32") for h in host]
    want = np.ascontiguousarray(oracle.eval_program(prog, host, [0.75], "f32")).view(np.uint32)
    assert S.salt_eval_route(prog, 3, 1, S.F32) == -1
    got = eval_bits(prog, dev, [0.75], "f32", n)      # first large call: interpreted
    assert np.array_equal(got, want)
    assert S.salt_eval_route(prog, 3, 1, S.F32) == -1
    got = eval_bits(prog, dev, [0.75], "f32", n)      # second: compiled, then run
    assert np.array_equal(got, want)
    assert S.salt_eval_route(prog, 3, 1, S.F32) == S.ROUTE_COMPILED
    got = eval_bits(prog, dev, [0.75], "f32", n)
    assert np.array_equal(got, want)
    # short calls never compile
    small = [T(S.LOAD, 1), T(S.LOAD, 0), T(S.MUL), T(S.LOAD, 0), T(S.ADD)]
    for _ in range(3):
        eval_bits(small, dev, [], "f32", 1000)
    assert S.salt_eval_route(small, 3, 0, S.F32) == -1


def test_graph_capture_before_and_after_loading():
    """A compiled kernel not yet loaded on the device is not loaded during
    stream capture (the call runs interpreted in the graph); once loaded,
    the captured launch is the compiled kernel. Every replay equals the
    eager result."""
    import torch

    S.salt_jit_set_mode(S.JIT_EXPLICIT)
    prog = [T(S.LOAD, 0), T(S.LOAD, 0), T(S.MUL), T(S.LOAD, 1), T(S.SUB)]     # a*a - b
    S.salt_jit_compile(prog, 2, 0, S.F64)
    n = 100003
    host = workloads.uniform(n, "f64", 6500, 2)
    dev = [to_dev(h, "f64") for h in host]
    want = np.ascontiguousarray(oracle.eval_program(prog, host, [], "f64")).view(np.uint64)
    for phase in range(2):
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        S.salt_eval(prog, dev, [], out)          # warm-up outside capture (loads it in phase 1)
        torch.cuda.synchronize()
        if phase == 0:
            # a second tree, compiled but never launched eagerly: first
            # seen inside the capture
            prog2 = [T(S.LOAD, 1), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 0), T(S.SUB)]
            S.salt_jit_compile(prog2, 2, 0, S.F64)
            want2 = np.ascontiguousarray(oracle.eval_program(prog2, host, [], "f64")).view(np.uint64)
            out2 = torch.empty(n, dtype=torch.float64, device="cuda")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            S.salt_eval(prog, dev, [], out)
            if phase == 0:
                S.salt_eval(prog2, dev, [], out2)
        for rep in range(3):
            out.zero_()
            if phase == 0:
                out2.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint64), want), (phase, rep)
            if phase == 0:
                assert np.array_equal(out2.cpu().numpy().view(np.uint64), want2), (phase, rep)
        del g


# ---- reduction pairs ----------------------------------------------------------

def reduce_value(px, py, dev, sc, n, cfg=None, result=None, ws=None):
    import torch

    if py is None:
        r = S.salt_nrm2_expr(px, dev, sc, n=n, config=cfg, result=result, ws=ws)
    else:
        r = S.salt_dot_expr(px, py, dev, sc, n=n, config=cfg, result=result, ws=ws)
    torch.cuda.synchronize()
    return r.item()


def oracle_close(got, px, py, host, sc, dtype, n):
    vx = oracle.widen(oracle.eval_program(px, host, sc, dtype, n=n), dtype)
    vy = vx if py is None else oracle.widen(oracle.eval_program(py, host, sc, dtype, n=n), dtype)
    ref, abs_sum = oracle.dot2(vx, vy)
    if py is None:
        return abs(got - np.sqrt(ref)) <= oracle.TOL[dtype] * np.sqrt(ref) + 1e-300
    return abs(got - ref) <= oracle.TOL[dtype] * abs_sum + 1e-300


@pytest.mark.parametrize("dtype", DTYPES)
def test_compiled_pairs_against_interpreter_and_oracle(dtype):
    rng = random.Random(5150 + len(dtype))
    Tt = S.salt_reduce_tile_elems(CODE[dtype])
    for trial in range(4):
        nops, nsc = rng.randint(1, 6), rng.randint(0, 2)
        px = rand_prog(rng, nops, nsc, rng.randint(1, 6))
        py = None if trial == 3 else rand_prog(rng, nops, nsc, rng.randint(1, 6))
        S.salt_jit_set_mode(S.JIT_EXPLICIT)
        S.salt_jit_compile_reduce(px, py, nops, nsc, CODE[dtype])
        route = S.salt_reduce_expr_route(px, py, nops, nsc, CODE[dtype])
        if route >= 0:
            continue                                   # drew a catalogue pair
        assert route == S.ROUTE_COMPILED
        sc = [rng.uniform(-2, 2) for _ in range(nsc)]
        for n in (1, 1000, Tt, Tt + 1, 3 * Tt + 11, 200003):
            off = rng.choice([0, 0, 1])
            host = workloads.uniform(n, dtype, 7000 + 10 * trial + n % 7, nops)
            dev = [to_dev(h, dtype, offset=off) for h in host]
            print("jit pair", trial, dtype, n, off, px, py, flush=True)
            S.salt_jit_set_mode(S.JIT_EXPLICIT)
            got = reduce_value(px, py, dev, sc, n)
            if py is not None:                         # the exchanged dot shares the kernel
                assert reduce_value(py, px, dev, sc, n) == got, (trial, n, "exchanged")
            S.salt_jit_set_mode(S.JIT_OFF)
            assert reduce_value(px, py, dev, sc, n) == got, (trial, dtype, n, off, "interpreter")
            assert oracle_close(got, px, py, host, sc, dtype, n), (trial, dtype, n, off)


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_compiled_pair_launch_shapes(dtype):
    """Every launch knob (chunks per burst clamped by the operand count,
    hints, grid) gives the interpreter's bits, for a pair of three and one
    of six operands, over several tiles and a ragged tail."""
    n = 5 * S.salt_reduce_tile_elems(CODE[dtype]) + 333
    host = workloads.uniform(n, dtype, 7300, 6)
    dev = [to_dev(h, dtype) for h in host]
    L = [T(S.LOAD, k) for k in range(6)]
    pairs = [([L[0], L[1], T(S.ADD), L[2], T(S.MUL)], [L[2], T(S.SCALAR, 0), T(S.SUB)]),
             ([L[0], L[1], T(S.MUL), L[2], L[3], T(S.MUL), T(S.ADD)], [L[4], L[5], T(S.SUB), L[0], T(S.MUL)])]
    for px, py in pairs:
        S.salt_jit_set_mode(S.JIT_OFF)
        want = reduce_value(px, py, dev, [0.5], n)
        wantn = reduce_value(px, None, dev, [0.5], n)
        S.salt_jit_set_mode(S.JIT_EXPLICIT)
        S.salt_jit_compile_reduce(px, py, 6, 1, CODE[dtype])
        S.salt_jit_compile_reduce(px, None, 6, 1, CODE[dtype])
        for unroll in (2, 4, 8, 16):
            for nt in (0, 1):
                for blocks in (0, 7, 256):
                    cfg = (unroll, nt, blocks)
                    assert reduce_value(px, py, dev, [0.5], n, cfg) == want, (px, cfg)
                    assert reduce_value(px, None, dev, [0.5], n, cfg) == wantn, (px, cfg)
        assert oracle_close(want, px, py, host, [0.5], dtype, n)


def test_automatic_mode_compiles_a_pair_on_its_second_large_call():
    S.salt_jit_set_mode(S.JIT_AUTO)
    # a pair no other test uses: dot((a - b) * c, a * alpha + c), binary32
    px = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.SUB), T(S.LOAD, 2), T(S.MUL)]
    py = [T(S.LOAD, 0), T(S.SCALAR, 0), T(S.MUL), T(S.LOAD, 2), T(S.ADD)]
    n = 1 << 18
    host = workloads.uniform(n, "f32", 7400, 3)
    dev = [to_dev(h, "f32") for h in host]
    assert S.salt_reduce_expr_route(px, py, 3, 1, S.F32) == -1
    r1 = reduce_value(px, py, dev, [1.5], n)                  # first large call: interpreted
    assert S.salt_reduce_expr_route(px, py, 3, 1, S.F32) == -1
    r2 = reduce_value(px, py, dev, [1.5], n)                  # second: compiled, then run
    assert S.salt_reduce_expr_route(px, py, 3, 1, S.F32) == S.ROUTE_COMPILED
    r3 = reduce_value(px, py, dev, [1.5], n)
    assert r1 == r2 == r3
    assert oracle_close(r1, px, py, host, [1.5], "f32", n)
    # short calls never compile, and an empty call stores zero
    small = [T(S.LOAD, 2), T(S.LOAD, 1), T(S.MUL)]
    for _ in range(3):
        reduce_value(small, None, dev, [], 1000)
    assert S.salt_reduce_expr_route(small, None, 3, 0, S.F32) == -1
    assert reduce_value(px, py, dev, [1.5], 0) == 0.0


def test_pair_graph_capture_before_and_after_loading():
    """A compiled pair not yet loaded on the device runs interpreted inside
    a capture; once loaded, the captured pass 1 is the compiled kernel. Every
    replay equals the eager result."""
    import torch

    S.salt_jit_set_mode(S.JIT_EXPLICIT)
    px = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 0), T(S.SUB)]      # a*b - a
    py = [T(S.LOAD, 1), T(S.LOAD, 1), T(S.ADD)]                              # b + b
    S.salt_jit_compile_reduce(px, py, 2, 0, S.F64)
    n = 300007
    host = workloads.uniform(n, "f64", 7500, 2)
    dev = [to_dev(h, "f64") for h in host]
    ws = S.workspace(n, S.F64)
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    for phase in range(2):
        if phase == 1:
            want = reduce_value(px, py, dev, [], n, result=res, ws=ws)    # loads the kernel
        else:
            S.salt_jit_set_mode(S.JIT_OFF)
            want = reduce_value(px, py, dev, [], n, result=res, ws=ws)
            S.salt_jit_set_mode(S.JIT_EXPLICIT)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            S.salt_dot_expr(px, py, dev, [], n=n, result=res, ws=ws)
        for rep in range(3):
            res.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert res.item() == want, (phase, rep)
        del g
    assert oracle_close(want, px, py, host, [], "f64", n)
