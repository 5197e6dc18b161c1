"""Trees outside the catalogue on their run-time compiled kernels: bit for
bit against the oracle and against the interpreter, in every element type,
at lengths spanning several tiles and ragged tails, aligned and not, in
place, under every launch shape; the automatic mode compiles a tree at its
second large call without changing a bit; a launch captured into a HIP
graph before the kernel is loaded runs interpreted and replays correctly."""
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
