"""Parity of the fused element-wise kernels with the CPU oracle: bit-exact,
through the C ABI, on seeded inputs spanning several tiles and a ragged tail,
for every catalogue tree, the generic interpreter, every element type, every
launch shape, unaligned views and in-place updates."""
from __future__ import annotations

import random

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from tests.gpu_util import first_mismatch, oracle_bits, to_dev, to_host_bits, empty

pytestmark = pytest.mark.gpu

DTYPES = ["f64", "f32", "bf16", "f16"]
# lengths: empty, tiny, around one and several tiles (256 lanes x U x V), ragged
LENGTHS = [0, 1, 7, 255, 4099, 65536 + 513, 300007]


def ops_for(prog):
    nops = 1 + max([t >> 8 for t in prog if t & 0xFF == S.LOAD], default=-1)
    nsc = 1 + max([t >> 8 for t in prog if t & 0xFF == S.SCALAR], default=-1)
    return nops, nsc


def run_case(prog, dtype, n, seed, offset=0, config=None, scalars=None):
    import torch

    nops, nsc = ops_for(prog)
    host = workloads.uniform(n, dtype, seed, max(nops, 1))[:nops]
    sc = scalars if scalars is not None else [workloads.alpha(seed + j) for j in range(nsc)]
    dev = [to_dev(h, dtype, offset=offset) for h in host]
    out = empty(n, dtype, offset=offset)
    print("case", [hex(t) for t in prog], dtype, n, seed, offset, config, flush=True)
    S.salt_eval(prog, dev, sc, out, config=config)
    torch.cuda.synchronize()
    want = oracle_bits(oracle.eval_program(prog, host, sc, dtype, n=n), dtype)
    got = to_host_bits(out, dtype)
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name", ["copy", "scale", "fig1", "axpy", "tree5", "abc", "t4", "t5"])
def test_catalogue_tree(name, dtype):
    prog = dict(S.salt_catalogue())[name]
    for k, n in enumerate(LENGTHS):
        run_case(prog, dtype, n, 100 + k)


@pytest.mark.parametrize("dtype", DTYPES)
def test_launch_shapes_do_not_change_bits(dtype):
    prog = dict(S.salt_catalogue())["tree5"]
    n = 123457
    for unroll in (1, 2, 4, 8):
        for nt in (0, 1):
            for blocks in (0, 1, 37, 1024):
                run_case(prog, dtype, n, 7, config=(unroll, nt, blocks))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("offset", [1, 3, 5])
def test_unaligned_views(dtype, offset):
    for name in ("fig1", "tree5"):
        run_case(dict(S.salt_catalogue())[name], dtype, 70001, 9, offset=offset)
    # the interpreter on unaligned data too
    T = S.token
    run_case([T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD), T(S.LOAD, 2), T(S.SUB)], dtype, 70001, 9, offset=offset)


@pytest.mark.parametrize("dtype", DTYPES)
def test_interpreter_random_programs(dtype):
    rng = random.Random(4242)
    T = S.token

    def build(leaves, nops, nsc):
        if leaves == 1:
            if nsc and rng.random() < 0.25:
                return [T(S.SCALAR, rng.randrange(nsc))]
            return [T(S.LOAD, rng.randrange(nops))]
        k = rng.randrange(1, leaves)
        return build(k, nops, nsc) + build(leaves - k, nops, nsc) + [T(rng.choice([S.ADD, S.SUB, S.MUL]))]

    done = 0
    while done < 40:
        nops, nsc = rng.randint(1, 8), rng.randint(0, 8)
        prog = build(rng.randint(1, 12), nops, nsc)
        try:
            S.salt_program_check(prog, nops, nsc)
        except S.SaltError:
            continue  # deeper than the stack limit
        n = rng.choice([1, 100, 4096 + 77, 50001])
        nops_used, nsc_used = ops_for(prog)
        run_case(prog, dtype, n, rng.randrange(1 << 20))
        done += 1


@pytest.mark.parametrize("dtype", DTYPES)
def test_interpreter_deep_stack_and_long_program(dtype):
    T = S.token
    # right-deep: a0 - (a1 - (a2 - ... (a6 - a7))) needs all 8 stack slots
    prog = [T(S.LOAD, k) for k in range(8)] + [T(S.SUB)] * 7
    assert S.salt_program_check(prog, 8, 0)[0] == 8
    run_case(prog, dtype, 33333, 5)
    # 63 tokens, left-deep, scalars mixed in
    prog = [T(S.LOAD, 0)]
    for k in range(31):
        prog += [T(S.SCALAR, k % 8) if k % 3 == 0 else T(S.LOAD, k % 8), T([S.ADD, S.SUB, S.MUL][k % 3])]
    run_case(prog, dtype, 20000, 6, scalars=[0.5, 1.5, -2.0, 0.25, 3.0, -0.75, 1.0, 2.0])


@pytest.mark.parametrize("dtype", DTYPES)
def test_in_place_update(dtype):
    import torch

    T = S.token
    n = 100003
    x, y = workloads.uniform(n, dtype, 31, 2)
    dx, dy = to_dev(x, dtype), to_dev(y, dtype)
    S.salt_axpy(1.75, dx, dy)
    torch.cuda.synchronize()
    want = oracle_bits(oracle.axpy(1.75, x, y, dtype), dtype)
    assert np.array_equal(to_host_bits(dy, dtype), want)
    # out aliases the first operand: a <- a*b - a (catalogue miss -> interpreter)
    a, b = workloads.uniform(n, dtype, 32, 2)
    da, db = to_dev(a, dtype), to_dev(b, dtype)
    prog = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 0), T(S.SUB)]
    S.salt_eval(prog, [da, db], [], da)
    torch.cuda.synchronize()
    want = oracle_bits(oracle.eval_program(prog, [a, b], [], dtype), dtype)
    assert np.array_equal(to_host_bits(da, dtype), want)


def test_special_values():
    """Signed zeros, subnormals, infinities, and a - a = +0, bit-exact."""
    import torch

    T = S.token
    for dtype, np_t in (("f64", np.float64), ("f32", np.float32)):
        vals = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 5e-324 if dtype == "f64" else 1e-45,
                         -2.5e-310 if dtype == "f64" else -3e-40, 1e300 if dtype == "f64" else 3e38,
                         np.finfo(np_t).max, np.finfo(np_t).tiny], dtype=np_t)
        a = np.tile(vals, 401)
        b = np.roll(a, 3)
        c = np.roll(a, 7)
        da, db, dc = (to_dev(v, dtype) for v in (a, b, c))
        for prog in (dict(S.salt_catalogue())["fig1"],
                     [T(S.LOAD, 0), T(S.LOAD, 0), T(S.SUB)],
                     [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 2), T(S.MUL)]):
            nops, _ = ops_for(prog)
            out = empty(len(a), dtype)
            S.salt_eval(prog, [da, db, dc][:nops], [], out)
            torch.cuda.synchronize()
            with np.errstate(all="ignore"):
                want = oracle.eval_program(prog, [a, b, c][:nops], [], dtype)
            got = to_host_bits(out, dtype)
            wb = oracle_bits(want, dtype)
            nan = np.isnan(want)
            assert np.array_equal(got[~nan], wb[~nan]), first_mismatch(got[~nan], wb[~nan])
            assert np.all(np.isnan(to_host_bits(out, dtype).view(np_t)[nan]))


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_16bit_rounding_edges(dtype):
    """Narrowing at the store: ties, overflow and gradual underflow, bit-exact
    against the oracle's rounding (products of chosen values)."""
    import torch

    T = S.token
    rng = np.random.Generator(np.random.PCG64(55))
    # all 16-bit patterns as a, and b = a value whose product hits ties
    allh = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    wid = oracle.widen(allh, dtype)
    finite = allh[np.isfinite(wid)]
    b = rng.choice(finite, len(finite))
    da, db = to_dev(finite, dtype), to_dev(b, dtype)
    for prog in ([T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL)], [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD)],
                 [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL)]):
        out = empty(len(finite), dtype)
        S.salt_eval(prog, [da, db], [1.0 + 2.0 ** -9], out)
        torch.cuda.synchronize()
        want = oracle.eval_program(prog, [finite, b], [1.0 + 2.0 ** -9], dtype)
        got = to_host_bits(out, dtype)
        w = oracle.widen(want, dtype)
        ok = ~np.isnan(w)
        assert np.array_equal(got[ok], want[ok]), first_mismatch(got[ok], want[ok])


def test_fig1_full_size_bit_exact():
    """The paper's Fig. 1 tree, FP64, n = 2^20, a, b, c ~ U[-1, 1) (seed 1109)."""
    import torch

    n = 1 << 20
    a, b, c = workloads.uniform(n, "f64", workloads.SEED_FIG1, 3)
    prog = dict(S.salt_catalogue())["fig1"]
    out = empty(n, "f64")
    S.salt_eval(prog, [to_dev(v, "f64") for v in (a, b, c)], [], out)
    torch.cuda.synchronize()
    want = oracle_bits(oracle.eval_program(prog, [a, b, c], [], "f64"), "f64")
    got = to_host_bits(out, "f64")
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_closed_form():
    import torch

    n = (1 << 22) + 3
    i = np.arange(n, dtype=np.float64)
    prog = dict(S.salt_catalogue())["fig1"]
    out = empty(n, "f64")
    S.salt_eval(prog, [to_dev(i, "f64"), to_dev(2 * i, "f64"), to_dev(i, "f64")], [], out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), 2 * i)


@pytest.mark.parametrize("dtype", DTYPES)
def test_programs_without_operands(dtype):
    """Trees of scalars only (no vector operand): every element is the same
    rounded value; aligned and unaligned outputs, ragged lengths."""
    T = S.token
    progs = [[T(S.SCALAR, 0)],
             [T(S.SCALAR, 0), T(S.SCALAR, 1), T(S.MUL)],
             [T(S.SCALAR, 1), T(S.SCALAR, 0), T(S.SUB), T(S.SCALAR, 2), T(S.ADD)]]
    for k, prog in enumerate(progs):
        for n in (1, 1000, 100003):
            for offset in (0, 1):
                run_case(prog, dtype, n, 7000 + k, offset=offset, scalars=[0.1, -3.75, 1e-3])
