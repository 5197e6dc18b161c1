"""Run-time compilation of trees outside the catalogue, on the host (hipRTC
needs no GPU): every element type compiles, the code object follows the
library's build rules (no packed binary32 instructions, no fused multiply-
add: every add, sub and mul stays one IEEE operation), catalogue trees are
not compiled again, and the route reflects what is cached. The same for
reduction pairs (dot and nrm2 of expressions), whose pass-1 kernels are
compiled from the library's own template. Nothing is loaded on a device or
launched here."""
from __future__ import annotations

import os
import random
import re
import shutil
import subprocess

import pytest

from paper_1109_1264_amd import salt as S

T = S.token
OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
DTS = [S.F64, S.F32, S.BF16, S.F16]


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
def explicit_mode():
    S.salt_jit_set_mode(S.JIT_EXPLICIT)
    yield
    S.salt_jit_set_mode(S.JIT_AUTO)


def disasm(code: bytes, tmp_path) -> str:
    p = tmp_path / "k.co"
    p.write_bytes(code)
    return subprocess.run([OBJDUMP, "-d", str(p)], capture_output=True, text=True, check=True).stdout


@pytest.mark.parametrize("dt", DTS)
def test_compiles_and_follows_the_build_rules(dt, tmp_path):
    # (a*b + c) * (a - e): multiplications next to additions, which
    # contraction would turn into fused multiply-adds
    prog = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 2), T(S.ADD),
            T(S.LOAD, 0), T(S.LOAD, 3), T(S.SUB), T(S.MUL)]
    assert S.salt_eval_route(prog, 4, 0, dt) == -1
    S.salt_jit_compile(prog, 4, 0, dt)
    assert S.salt_eval_route(prog, 4, 0, dt) == S.ROUTE_COMPILED
    code = S.salt_jit_code(prog, 4, 0, dt)
    assert code[:4] == b"\x7fELF"
    if not os.path.exists(OBJDUMP):
        pytest.skip("llvm-objdump not installed")
    asm = disasm(code, tmp_path)
    # the library's element-wise template, in six variants (1, 2, 4 chunks
    # per lane; cached and streaming)
    assert len(set(re.findall(r"_ZN4salt11k_eval_tree\w+", asm))) == 6
    assert not re.search(r"\bv_pk_(add|mul|fma)_f32\b", asm), "packed binary32 instruction"
    assert not re.search(r"\bv_(fma|fmac|mad|mac)_(f32|f64|legacy)", asm), "contracted multiply-add"
    assert re.search(r"\bv_mul_f(32|64)", asm) and re.search(r"\bv_(add|sub)_f(32|64)", asm)


def test_random_trees_compile_and_catalogue_trees_are_not_recompiled():
    rng = random.Random(77)
    for trial in range(6):
        nops, nsc = rng.randint(1, 8), rng.randint(0, 3)
        prog = rand_prog(rng, nops, nsc, rng.randint(2, 7))
        dt = DTS[trial % 4]
        S.salt_jit_compile(prog, nops, nsc, dt)
        r = S.salt_eval_route(prog, nops, nsc, dt)
        assert r == S.ROUTE_COMPILED or r >= 0, (trial, prog, r)
    fig1 = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.LOAD, 2), T(S.SUB), T(S.ADD)]
    S.salt_jit_compile(fig1, 3, 0, S.F64)          # nothing to do
    assert S.salt_eval_route(fig1, 3, 0, S.F64) == 2
    assert S.salt_jit_code(fig1, 3, 0, S.F64) == b""


def test_modes_and_errors():
    prog = [T(S.LOAD, 1), T(S.LOAD, 0), T(S.SUB), T(S.SCALAR, 0), T(S.MUL)]
    S.salt_jit_compile(prog, 2, 1, S.F32)
    assert S.salt_eval_route(prog, 2, 1, S.F32) == S.ROUTE_COMPILED
    S.salt_jit_set_mode(S.JIT_OFF)
    assert S.salt_eval_route(prog, 2, 1, S.F32) == -1      # the interpreter while off
    with pytest.raises(S.SaltError):
        S.salt_jit_set_mode(3)
    with pytest.raises(S.SaltError):
        S.salt_jit_compile([T(S.ADD)], 1, 0, S.F32)        # malformed program
    with pytest.raises(S.SaltError):
        S.salt_jit_compile(prog, 2, 1, 9)                   # unknown dtype


# A dot pair outside the reduction catalogue: dot(a*b + c, e*alpha).
PAIR_X = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 2), T(S.ADD)]
PAIR_Y = [T(S.LOAD, 3), T(S.SCALAR, 0), T(S.MUL)]


@pytest.mark.parametrize("dt", DTS)
def test_reduction_pairs_compile(dt, tmp_path):
    assert S.salt_reduce_expr_route(PAIR_X, PAIR_Y, 4, 1, dt) == -1
    S.salt_jit_compile_reduce(PAIR_X, PAIR_Y, 4, 1, dt)
    assert S.salt_reduce_expr_route(PAIR_X, PAIR_Y, 4, 1, dt) == S.ROUTE_COMPILED
    # the dot with its programs exchanged shares the kernel (same bits)
    assert S.salt_reduce_expr_route(PAIR_Y, PAIR_X, 4, 1, dt) == S.ROUTE_COMPILED
    # so does any operand and scalar numbering of the same pair
    rx = [T(S.LOAD, 2), T(S.LOAD, 0), T(S.MUL), T(S.LOAD, 3), T(S.ADD)]
    ry = [T(S.LOAD, 1), T(S.SCALAR, 1), T(S.MUL)]
    assert S.salt_reduce_expr_route(rx, ry, 4, 2, dt) == S.ROUTE_COMPILED
    code = S.salt_jit_code_reduce(PAIR_X, PAIR_Y, 4, 1, dt)
    assert code[:4] == b"\x7fELF"
    assert S.salt_jit_code_reduce(PAIR_Y, PAIR_X, 4, 1, dt) == code
    # six pass-1 variants (2, 4, 8 chunks per burst; cached and streaming)
    syms = set(re.findall(rb"_ZN4salt13k_reduce_tree[A-Za-z0-9_]+", code))
    assert len(syms) == 6, syms
    if not os.path.exists(OBJDUMP):
        pytest.skip("llvm-objdump not installed")
    asm = disasm(code, tmp_path)
    assert not re.search(r"\bv_pk_(add|mul|fma)_f32\b", asm), "packed binary32 instruction"


def test_reduction_pair_norm_and_catalogue():
    nx = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.LOAD, 2), T(S.SUB), T(S.MUL)]     # a * (b - c)
    assert S.salt_reduce_expr_route(nx, None, 3, 0, S.F32) == -1
    S.salt_jit_compile_reduce(nx, None, 3, 0, S.F32)
    assert S.salt_reduce_expr_route(nx, None, 3, 0, S.F32) == S.ROUTE_COMPILED
    assert S.salt_reduce_expr_route(nx, None, 3, 0, S.F64) == -1          # not compiled for binary64
    # nrm2(P) and dot(P, P) are different kernels
    assert S.salt_reduce_expr_route(nx, nx, 3, 0, S.F32) == -1
    # a pair with an ahead-of-time kernel is not compiled again
    s, d = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD)], [T(S.LOAD, 0), T(S.LOAD, 1), T(S.SUB)]
    S.salt_jit_compile_reduce(s, d, 2, 0, S.F64)
    assert S.salt_reduce_expr_route(s, d, 2, 0, S.F64) == 0
    assert S.salt_jit_code_reduce(s, d, 2, 0, S.F64) == b""
    S.salt_jit_set_mode(S.JIT_OFF)
    assert S.salt_reduce_expr_route(nx, None, 3, 0, S.F32) == -1           # the interpreter while off
    S.salt_jit_set_mode(S.JIT_EXPLICIT)
    with pytest.raises(S.SaltError):
        S.salt_jit_compile_reduce(nx, [T(S.SUB)], 3, 0, S.F32)              # malformed second program
    with pytest.raises(S.SaltError):
        S.salt_jit_compile_reduce(nx, None, 3, 0, 9)                        # unknown dtype
    with pytest.raises(S.SaltError):
        S.salt_reduce_expr_route(nx, None, 3, 0, 9)


def test_concurrent_compiles_of_one_key():
    """Threads compiling the same tree or pair at once: one compiles, the
    others wait for it; all see the same code object."""
    import threading

    prog = [T(S.LOAD, 2), T(S.LOAD, 0), T(S.SUB), T(S.LOAD, 1), T(S.MUL), T(S.SCALAR, 0), T(S.ADD)]
    px = [T(S.LOAD, 0), T(S.LOAD, 2), T(S.MUL), T(S.LOAD, 1), T(S.SUB)]
    errors, codes = [], []

    def work(k):
        try:
            if k % 2:
                S.salt_jit_compile(prog, 3, 1, S.BF16)
                codes.append(("e", S.salt_jit_code(prog, 3, 1, S.BF16)))
            else:
                S.salt_jit_compile_reduce(px, None, 3, 0, S.F32)
                codes.append(("r", S.salt_jit_code_reduce(px, None, 3, 0, S.F32)))
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(6)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for kind in ("e", "r"):
        got = [c for k, c in codes if k == kind]
        assert len(got) == 3 and got[0][:4] == b"\x7fELF" and all(c == got[0] for c in got)
