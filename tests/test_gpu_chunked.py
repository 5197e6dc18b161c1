"""Large element-wise calls of trees reading three or more operands run as
a sequence of launches over 128 MiB chunks per operand (the last one taking
the remainder). Every element must be what one launch computes: bit-exact
against the oracle over whole arrays spanning several chunks and a ragged
last chunk, aligned and not, in place, for catalogue trees, a compiled tree
and the interpreter."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from tests.gpu_util import CODE, empty, first_mismatch, oracle_bits, to_dev, to_host_bits

pytestmark = pytest.mark.gpu
T = S.token
CHUNK_BYTES = 128 << 20
ES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}


def length(dtype, extra=12345):
    """Two whole chunks and a third one with a remainder."""
    c = CHUNK_BYTES // ES[dtype]
    return 2 * c + c // 3 + extra


def run(prog, host, sc, dtype, n, offset=0):
    import torch

    dev = [to_dev(h, dtype, offset=offset) for h in host]
    out = empty(n, dtype, offset=offset)
    print("chunked", dtype, n, offset, prog, flush=True)
    S.salt_eval(prog, dev, sc, out)
    torch.cuda.synchronize()
    got = to_host_bits(out, dtype)
    del dev, out
    torch.cuda.empty_cache()
    return got


@pytest.mark.parametrize("dtype,offset", [("f64", 0), ("f64", 1), ("bf16", 0), ("f32", 1)])
def test_catalogue_trees(dtype, offset):
    cat = dict(S.salt_catalogue())
    n = length(dtype)
    for name in ("fig1", "tree5"):
        prog = cat[name]
        k = 1 + max(t >> 8 for t in prog if t & 0xFF == S.LOAD)
        host = workloads.uniform(n, dtype, 9100 + k, k)
        want = oracle_bits(oracle.eval_program(prog, host, [], dtype), dtype)
        got = run(prog, host, [], dtype, n, offset)
        assert np.array_equal(got, want), (name, dtype, offset, first_mismatch(got, want))


def test_in_place():
    """d = alpha*(a + b) - c*d with the output in operand 3's place."""
    import torch

    dtype = "f32"
    n = length(dtype, extra=5)
    t4 = dict(S.salt_catalogue())["t4"]
    host = workloads.uniform(n, dtype, 9200, 4)
    want = oracle_bits(oracle.eval_program(t4, host, [1.5], dtype), dtype)
    dev = [to_dev(h, dtype) for h in host]
    S.salt_eval(t4, dev, [1.5], dev[3])
    torch.cuda.synchronize()
    got = to_host_bits(dev[3], dtype)
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("mode", ["compiled", "interpreter"])
def test_tree_outside_the_catalogue(mode):
    dtype = "bf16"
    n = length(dtype, extra=77)
    prog = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD), T(S.LOAD, 2), T(S.MUL), T(S.SCALAR, 0), T(S.SUB)]
    host = workloads.uniform(n, dtype, 9300, 3)
    want = oracle_bits(oracle.eval_program(prog, host, [0.625], dtype), dtype)
    try:
        if mode == "compiled":
            S.salt_jit_set_mode(S.JIT_EXPLICIT)
            S.salt_jit_compile(prog, 3, 1, CODE[dtype])
        else:
            S.salt_jit_set_mode(S.JIT_OFF)
        got = run(prog, host, [0.625], dtype, n)
    finally:
        S.salt_jit_set_mode(S.JIT_AUTO)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_chunked_call_in_a_graph():
    """A chunked call captured into a HIP graph replays the same bits, with
    eager work and synchronisations between the replays."""
    import torch

    dtype = "f64"
    n = length(dtype, extra=3)
    fig1 = dict(S.salt_catalogue())["fig1"]
    assert S.salt_eval_chunking(3, n, S.F64)[1] == 2
    host = workloads.uniform(n, dtype, 9400, 3)
    dev = [to_dev(h, dtype) for h in host]
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    S.salt_eval(fig1, dev, [], out)                  # eager first (loads nothing new, sets the tuned path)
    torch.cuda.synchronize()
    want = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        S.salt_eval(fig1, dev, [], out)
    for rep in range(3):
        out.zero_()
        torch.randn(1 << 20, device="cuda").mul_(3.0).sum()     # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int64), want.view(torch.int64)), rep
    del g
    got = out.cpu().numpy().view(np.uint64)
    ref = oracle_bits(oracle.eval_program(fig1, host, [], dtype), dtype)
    assert np.array_equal(got, ref), first_mismatch(got, ref)
