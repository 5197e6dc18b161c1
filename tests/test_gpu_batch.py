"""Batched launches against the oracle and against single calls: every
item's element-wise output is bit-exact, every item's dot has exactly the
bits salt_dot gives for it alone (and is within tolerance of Dot2), for
direct launches, every launch shape, and repeated HIP-graph replays."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from paper_1109_1264_amd.batch import Batch
from tests.gpu_util import CODE, first_mismatch, oracle_bits, to_dev, to_host_bits, empty

pytestmark = pytest.mark.gpu

T = S.token
ABC = [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL), T(S.LOAD, 1), T(S.LOAD, 2), T(S.SUB), T(S.ADD)]


def make_batch(dtype, lengths, seed, dot_every=1, out_every=1, offsets=None):
    import torch

    items, host = [], []
    for i, n in enumerate(lengths):
        a, b, c = workloads.uniform(int(n), dtype, seed + i, 3)
        al = workloads.alpha(seed + i)
        off = 0 if offsets is None else offsets[i % len(offsets)]
        da, db, dc = (to_dev(v, dtype, offset=off) for v in (a, b, c))
        out = empty(int(n), dtype, offset=off) if i % out_every == 0 else None
        dot = (torch.empty(1, dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
               if i % dot_every == 0 else None)
        items.append({"n": int(n), "operands": [da, db, dc], "scalars": [al], "out": out, "dot_out": dot})
        host.append((a, b, c, al))
    return items, host


def check(items, host, dtype, alone_dot=True):
    import torch

    torch.cuda.synchronize()
    for i, (it, (a, b, c, al)) in enumerate(zip(items, host)):
        if it["out"] is not None:
            want = oracle_bits(oracle.eval_program(ABC, [a, b, c], [al], dtype), dtype)
            got = to_host_bits(it["out"], dtype)
            assert np.array_equal(got, want), (i, it["n"], first_mismatch(got, want))
        if it["dot_out"] is not None:
            got = float(it["dot_out"].item())
            ref, abs_sum = oracle.dot2(oracle.widen(a, dtype), oracle.widen(b, dtype))
            assert abs(got - ref) <= oracle.TOL[dtype] * abs_sum, (i, it["n"], got, ref)
            if alone_dot:
                r = S.salt_dot(it["operands"][0], it["operands"][1], n=it["n"])
                torch.cuda.synchronize()
                assert float(r.item()) == got, (i, it["n"], float(r.item()), got)


def ragged_lengths(dtype, count=60, seed=1):
    Tt = S.salt_reduce_tile_elems(CODE[dtype])
    fixed = [0, 1, 7, 63, Tt - 1, Tt, Tt + 1, 2 * Tt + 5]
    rnd = workloads.batch_lengths(count - len(fixed), seed=seed, median=2048, hi=1 << 17)
    return fixed + [int(v) for v in rnd]


@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16", "f16"])
def test_batch_matches_oracle_and_single_calls(dtype):
    items, host = make_batch(dtype, ragged_lengths(dtype), 500)
    b = Batch(ABC, items, CODE[dtype])
    print("batch", dtype, len(items), "items", b.tiles, "tiles", flush=True)
    b.launch()
    check(items, host, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch_mixed_outputs_dots_and_alignment(dtype):
    items, host = make_batch(dtype, ragged_lengths(dtype, 40, seed=3), 700, dot_every=2, out_every=3,
                             offsets=[0, 1, 3])
    b = Batch(ABC, items, CODE[dtype])
    b.launch()
    check(items, host, dtype)


def test_batch_launch_shapes_same_bits():
    import torch

    dtype = "f32"
    items, host = make_batch(dtype, ragged_lengths(dtype, 30, seed=5), 900)
    b = Batch(ABC, items, CODE[dtype])
    b.launch()
    torch.cuda.synchronize()
    ref_out = [to_host_bits(it["out"], dtype) for it in items]
    ref_dot = [float(it["dot_out"].item()) for it in items]
    for unroll in (2, 4, 8):
        for nt in (0, 1):
            for blocks in (0, 1, 7, 256):
                for it in items:
                    it["out"].zero_()
                b.launch(config=(unroll, nt, blocks))
                torch.cuda.synchronize()
                for i, it in enumerate(items):
                    assert np.array_equal(to_host_bits(it["out"], dtype), ref_out[i])
                    assert float(it["dot_out"].item()) == ref_dot[i], (unroll, nt, blocks, i)


def test_graph_replays():
    """Replay the captured graph several times with eager work in between;
    every replay must reproduce the eager launch exactly."""
    import torch

    dtype = "f32"
    lengths = [int(v) for v in workloads.batch_lengths(300, seed=7, hi=1 << 16)]
    items, host = make_batch(dtype, lengths, 1300)
    b = Batch(ABC, items, CODE[dtype])
    b.launch()
    torch.cuda.synchronize()
    ref_out = [to_host_bits(it["out"], dtype) for it in items]
    ref_dot = [float(it["dot_out"].item()) for it in items]
    check(items, host, dtype, alone_dot=False)
    g = b.graph()
    for rep in range(4):
        for it in items:
            it["out"].fill_(0.0)
            it["dot_out"].fill_(-1.0)
        scratch = torch.randn(1 << 20, device="cuda")
        scratch.mul_(2.0).sum()                       # unrelated eager work
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for i, it in enumerate(items):
            assert np.array_equal(to_host_bits(it["out"], dtype), ref_out[i]), (rep, i)
            assert float(it["dot_out"].item()) == ref_dot[i], (rep, i)
    g.close()


def test_c4_shape_small():
    """The batched workload's shape (lognormal lengths, FP32, alpha_k a_k +
    (b_k - c_k) with dot(a_k, b_k)) on 512 instances."""
    dtype = "f32"
    lengths = [int(v) for v in workloads.batch_lengths(512, seed=workloads.SEED_BATCHED)]
    items, host = make_batch(dtype, lengths, workloads.SEED_BATCHED)
    b = Batch(ABC, items, CODE[dtype])
    b.graph().launch()
    check(items, host, dtype, alone_dot=False)


def test_item_with_more_partials_than_combine_lanes():
    """An item with more than 1024 tiles: the one-wave combine of the batched
    path and the 1024-lane pass 2 of salt_dot must still agree bit for bit."""
    import torch

    dtype = "bf16"
    Tt = S.salt_reduce_tile_elems(CODE[dtype])
    lengths = [1030 * Tt + 17, 5, Tt * 3]
    items = []
    for i, n in enumerate(lengths):
        a, b, c = workloads.uniform_device(n, dtype, 77 + i, 3)
        items.append({"n": n, "operands": [a, b, c], "scalars": [0.75], "out": None,
                      "dot_out": torch.empty(1, dtype=torch.float32, device="cuda")})
    bt = Batch(ABC, items, CODE[dtype])
    bt.launch()
    torch.cuda.synchronize()
    for it in items:
        r = S.salt_dot(it["operands"][0], it["operands"][1])
        torch.cuda.synchronize()
        assert float(r.item()) == float(it["dot_out"].item()), it["n"]


def test_c4_full_size():
    """The batched workload at its full size: 4096 instances, lognormal
    lengths (median 4096, clipped 64..2^20, about 50.6 M elements), FP32,
    alpha_k a_k + (b_k - c_k) and dot(a_k, b_k), one graph launch with the
    tuned knobs; every output bit-exact and every dot within tolerance of the
    oracle, and every dot with the bits of the same item run alone."""
    dtype = "f32"
    lengths = [int(v) for v in workloads.batch_lengths(4096, seed=workloads.SEED_BATCHED)]
    assert 50_000_000 < sum(lengths) < 51_000_000
    items, host = make_batch(dtype, lengths, workloads.SEED_BATCHED)
    b = Batch(ABC, items, CODE[dtype])
    g = b.graph()
    print("c4 full size: %d items, %d elements" % (len(items), sum(lengths)), flush=True)
    g.launch()
    check(items, host, dtype, alone_dot=True)
    g.close()
    b.close()


# ---- trees outside the catalogue (batched kernels compiled at plan creation) --

L0, L1, L2, L3, L4, L5 = (T(S.LOAD, k) for k in range(6))
SC0 = T(S.SCALAR, 0)
ADD, SUB, MUL = T(S.ADD), T(S.SUB), T(S.MUL)
COMPILED_TREES = [
    ([L0, L1, MUL, L2, ADD, SC0, MUL], 3, 1),                                  # (a*b + c)*alpha
    ([L0, L1, SUB, L0, MUL, L2, L3, MUL, SUB], 4, 0),                          # (a - b)*a - c*e
    ([L0, L1, ADD, L2, L3, ADD, MUL, L4, L5, SUB, MUL, SC0, SUB], 6, 1),       # six operands
]


def make_tree_batch(prog, nops, nsc, dtype, lengths, seed, dot_every=2, offsets=(0,)):
    import torch

    items, host = [], []
    for i, n in enumerate(lengths):
        ops = workloads.uniform(int(n), dtype, seed + i, nops)
        sc = [workloads.alpha(seed + i)] * nsc
        off = offsets[i % len(offsets)]
        dev = [to_dev(v, dtype, offset=off) for v in ops]
        out = empty(int(n), dtype, offset=off)
        dot = (torch.empty(1, dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")
               if i % dot_every == 0 else None)
        items.append({"n": int(n), "operands": dev, "scalars": sc, "out": out, "dot_out": dot})
        host.append((ops, sc))
    return items, host


def check_tree_batch(prog, items, host, dtype):
    import torch

    torch.cuda.synchronize()
    for i, (it, (ops, sc)) in enumerate(zip(items, host)):
        want = oracle_bits(oracle.eval_program(prog, ops, sc, dtype), dtype)
        got = to_host_bits(it["out"], dtype)
        assert np.array_equal(got, want), (i, it["n"], first_mismatch(got, want))
        if it["dot_out"] is not None:
            got_dot = float(it["dot_out"].item())
            r = S.salt_dot(it["operands"][0], it["operands"][1], n=it["n"])
            torch.cuda.synchronize()
            assert float(r.item()) == got_dot, (i, it["n"])
            ref, abs_sum = oracle.dot2(oracle.widen(ops[0], dtype), oracle.widen(ops[1], dtype))
            assert abs(got_dot - ref) <= oracle.TOL[dtype] * abs_sum, (i, it["n"], got_dot, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_compiled_tree_batches(dtype):
    """Each tree outside the catalogue, batched over ragged and unaligned
    items with a fused dot on every other item: bit-exact against the oracle,
    dots with the bits of salt_dot alone; then a graph of the same plan
    replays the same bits."""
    import torch

    for k, (prog, nops, nsc) in enumerate(COMPILED_TREES):
        assert S.salt_program_route(prog, nops, nsc) == -1
        lengths = ragged_lengths(dtype, 24, seed=11 + k)
        items, host = make_tree_batch(prog, nops, nsc, dtype, lengths, 2100 + 100 * k, offsets=(0, 0, 1))
        print("compiled tree batch", dtype, k, len(items), "items", flush=True)
        b = Batch(prog, items, CODE[dtype])
        b.launch()
        check_tree_batch(prog, items, host, dtype)
        ref_out = [to_host_bits(it["out"], dtype) for it in items]
        ref_dot = [None if it["dot_out"] is None else float(it["dot_out"].item()) for it in items]
        g = b.graph()
        for rep in range(2):
            for it in items:
                it["out"].zero_()
                if it["dot_out"] is not None:
                    it["dot_out"].fill_(-1.0)
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for i, it in enumerate(items):
                assert np.array_equal(to_host_bits(it["out"], dtype), ref_out[i]), (k, rep, i)
                if ref_dot[i] is not None:
                    assert float(it["dot_out"].item()) == ref_dot[i], (k, rep, i)
        g.close()
        b.close()


def test_compiled_tree_batch_launch_shapes():
    """Every launch knob of a compiled batched tree gives the same bits."""
    import torch

    dtype = "f32"
    prog, nops, nsc = COMPILED_TREES[2]
    items, host = make_tree_batch(prog, nops, nsc, dtype, ragged_lengths(dtype, 20, seed=21), 2600)
    b = Batch(prog, items, CODE[dtype])
    b.launch()
    check_tree_batch(prog, items, host, dtype)
    ref_out = [to_host_bits(it["out"], dtype) for it in items]
    ref_dot = [None if it["dot_out"] is None else float(it["dot_out"].item()) for it in items]
    for unroll in (2, 4, 8):
        for nt in (0, 1):
            for blocks in (0, 1, 7, 256):
                for it in items:
                    it["out"].zero_()
                b.launch(config=(unroll, nt, blocks))
                torch.cuda.synchronize()
                for i, it in enumerate(items):
                    assert np.array_equal(to_host_bits(it["out"], dtype), ref_out[i]), (unroll, nt, blocks, i)
                    if ref_dot[i] is not None:
                        assert float(it["dot_out"].item()) == ref_dot[i], (unroll, nt, blocks, i)
    b.close()


def test_long_list_split_into_ranges():
    """A plan whose tiles hold more than twice 128 MiB per operand runs as
    several launches over consecutive ranges of its list, the dots' combine
    after the last: outputs bit-exact against the oracle, every dot with the
    bits of salt_dot alone, the same bits from a graph of the plan."""
    import torch

    dtype = "bf16"
    lengths = [(1 << 24) + 17 * i for i in range(9)] + [5, 70000]   # 288 MiB per operand: two ranges
    items, host = make_batch(dtype, lengths, 3300, dot_every=2)
    b = Batch(ABC, items, CODE[dtype])
    print("long batch", b.tiles, "tiles", flush=True)
    b.launch()
    check(items, host, dtype)
    ref_out = [to_host_bits(it["out"], dtype) for it in items]
    ref_dot = [None if it["dot_out"] is None else float(it["dot_out"].item()) for it in items]
    g = b.graph()
    for it in items:
        it["out"].zero_()
        if it["dot_out"] is not None:
            it["dot_out"].fill_(-1.0)
    torch.cuda.synchronize()
    g.launch()
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        assert np.array_equal(to_host_bits(it["out"], dtype), ref_out[i]), i
        if ref_dot[i] is not None:
            assert float(it["dot_out"].item()) == ref_dot[i], i
    g.close()
    b.close()
