"""Host-side checks of the batched planner (no GPU: planning makes no HIP
call; nothing here is uploaded or launched)."""
from __future__ import annotations

import ctypes

import pytest

from paper_1109_1264_amd import salt as S

T = S.token
ABC = [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL), T(S.LOAD, 1), T(S.LOAD, 2), T(S.SUB), T(S.ADD)]


def make_items(specs):
    arr = (S.BatchItem * max(1, len(specs)))()
    for i, (n, ops, out, dot) in enumerate(specs):
        arr[i].n = n
        for k, p in enumerate(ops):
            arr[i].operands[k] = p
        arr[i].scalars[0] = 1.5
        arr[i].out = out
        arr[i].dot_out = dot
    return arr


def plan(prog, specs, dtype=S.F32, nops=3, nsc=1):
    L = S.lib()
    arr = make_items(specs)
    parr, plen = S._prog(prog)
    h = ctypes.c_void_p()
    st = L.salt_batch_plan_create(parr, plen, nops, nsc, arr, len(specs), dtype, ctypes.byref(h))
    return st, h


def info(h):
    tb, wb, t = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int64()
    assert S.lib().salt_batch_plan_info(h, ctypes.byref(tb), ctypes.byref(wb), ctypes.byref(t)) == S.OK
    return tb.value, wb.value, t.value


def test_tiles_table_and_workspace_sizes():
    Tf = S.salt_reduce_tile_elems(S.F32)
    base = 1 << 32
    specs = [(0, [base, base + 2**24, base + 2**25], base + 2**26, None),
             (1, [base, base + 2**24, base + 2**25], base + 2**26, base + 2**30),
             (Tf, [base, base + 2**24, base + 2**25], base + 2**26, None),
             (Tf + 1, [base, base + 2**24, base + 2**25], base + 2**26, base + 2**30 + 8)]
    st, h = plan(ABC, specs)
    assert st == S.OK, S.lib().salt_last_error()
    tb, wb, tiles = info(h)
    assert tiles == 0 + 1 + 1 + 2
    # descriptors, then the execution list (item, tile) pairs
    assert tb == ((4 * 256 + 8 * tiles + 255) // 256) * 256
    assert wb == 8 * tiles
    S.lib().salt_batch_plan_destroy(h)
    # without any dot: no workspace
    st, h = plan(ABC, [(s[0], s[1], s[2], None) for s in specs])
    assert st == S.OK and info(h)[1] == 0
    S.lib().salt_batch_plan_destroy(h)
    # empty batch
    st, h = plan(ABC, [])
    assert st == S.OK and info(h) == (0, 0, 0)
    S.lib().salt_batch_plan_destroy(h)


def test_planner_rejects():
    base = 1 << 32
    good = [base, base + 2**24, base + 2**25]
    # a tree outside the catalogue while run-time compilation is off
    prog = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD), T(S.LOAD, 2), T(S.SUB)]
    S.salt_jit_set_mode(S.JIT_OFF)
    try:
        assert plan(prog, [(10, good, base + 2**26, None)], nsc=0)[0] == S.ERR_UNSUPPORTED
    finally:
        S.salt_jit_set_mode(S.JIT_AUTO)
    # dot whose operands are not the first two read
    prog = [T(S.SCALAR, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 0), T(S.LOAD, 2), T(S.SUB), T(S.ADD)]
    st, _ = plan(prog, [(10, good, base + 2**26, base + 2**30)])
    assert st == S.ERR_UNSUPPORTED
    # ... fine without the dot
    st, h = plan(prog, [(10, good, base + 2**26, None)])
    assert st == S.OK
    S.lib().salt_batch_plan_destroy(h)
    # null operand, negative n, partial overlap, bad dtype
    assert plan(ABC, [(10, [base, 0, base + 2**25], base + 2**26, None)])[0] == S.ERR_ARG
    assert plan(ABC, [(-1, good, base + 2**26, None)])[0] == S.ERR_ARG
    assert plan(ABC, [(10, good, base + 4, None)])[0] == S.ERR_ARG
    assert plan(ABC, [(10, good, base + 2**26, None)], dtype=9)[0] == S.ERR_ARG
    assert plan(ABC[:-1], [(10, good, base + 2**26, None)])[0] == S.ERR_PROGRAM


def test_launch_requires_upload():
    base = 1 << 32
    st, h = plan(ABC, [(10, [base, base + 2**24, base + 2**25], base + 2**26, None)])
    assert st == S.OK
    assert S.lib().salt_batch_launch(h, None, 0, None, None) == S.ERR_ARG
    assert b"uploaded" in S.lib().salt_last_error()
    assert S.lib().salt_batch_upload(h, None, 1 << 20, None) == S.ERR_ARG
    assert S.lib().salt_batch_upload(h, base + 16, 1 << 20, None) == S.ERR_ARG   # misaligned table
    assert S.lib().salt_batch_upload(h, base, 16, None) == S.ERR_ARG             # too small
    S.lib().salt_batch_plan_destroy(h)


def test_planner_compiles_trees_outside_the_catalogue():
    """A tree without ahead-of-time kernels gets its batched kernels compiled
    at plan creation (no GPU needed), with and without the fused dot; the
    plan's table and workspace are those of any other tree."""
    base = 1 << 32
    good = [base, base + 2**24, base + 2**25]
    prog = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 2), T(S.ADD), T(S.SCALAR, 0), T(S.MUL)]
    assert S.salt_program_route(prog, 3, 1) == -1
    Tf = S.salt_reduce_tile_elems(S.F32)
    for dot in (None, base + 2**30):
        st, h = plan(prog, [(Tf + 3, good, base + 2**26, dot)])
        assert st == S.OK, S.lib().salt_last_error()
        tb, wb, tiles = info(h)
        assert tiles == 2 and wb == (16 if dot else 0)
        S.lib().salt_batch_plan_destroy(h)
    # a dot still needs operands 0 and 1 read first
    prog2 = [T(S.LOAD, 2), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 0), T(S.ADD)]
    assert plan(prog2, [(10, good, base + 2**26, base + 2**30)], nsc=0)[0] == S.ERR_UNSUPPORTED
