"""C ABI checks that need no GPU: the library loads, exports every entry
point of include/salt.h, and rejects bad programs and arguments before
enqueuing anything (so none of these calls reaches the HIP runtime).

No call here passes validation with n > 0: fake addresses are only used in
calls that must be rejected.
"""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_1109_1264_amd import salt as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
T = S.token
FIG1 = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.LOAD, 2), T(S.SUB), T(S.ADD)]


@pytest.fixture(scope="module")
def L():
    return S.lib()


def header_functions():
    src = open(os.path.join(ROOT, "include", "salt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(salt_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_function(L):
    names = header_functions()
    assert "salt_eval" in names and "salt_dot" in names and len(names) >= 18
    for name in names:
        assert hasattr(L, name), name


def test_version_and_status_strings(L):
    assert S.salt_version() >= 10000
    for s in range(6):
        assert L.salt_status_string(s)
    assert L.salt_status_string(99) == b"unknown status"


@pytest.mark.parametrize("prog,nops,nsc,code", [
    ([], 1, 0, S.ERR_PROGRAM),                                  # empty
    ([T(S.LOAD, 0)] * 65, 1, 0, S.ERR_PROGRAM),                 # too long
    ([T(S.ADD)], 1, 0, S.ERR_PROGRAM),                          # underflow
    ([T(S.LOAD, 0), T(S.SUB)], 1, 0, S.ERR_PROGRAM),            # underflow
    ([T(S.LOAD, 0), T(S.LOAD, 0)], 1, 0, S.ERR_PROGRAM),        # two values left
    ([T(S.LOAD, 1)], 1, 0, S.ERR_PROGRAM),                      # operand out of range
    ([T(S.SCALAR, 0)], 1, 0, S.ERR_PROGRAM),                    # scalar out of range
    ([T(S.LOAD, 0), T(S.LOAD, 0), T(S.ADD, 1)], 1, 0, S.ERR_PROGRAM),  # binary with arg
    ([9], 1, 0, S.ERR_PROGRAM),                                 # unknown opcode
    ([0], 1, 0, S.ERR_PROGRAM),
    ([T(S.LOAD, 0)] * 9 + [T(S.ADD)] * 8, 1, 0, S.ERR_PROGRAM),  # stack depth 9 > 8
    ([T(S.LOAD, 0)], 9, 0, S.ERR_ARG),                          # too many operands
    ([T(S.LOAD, 0)], 1, 9, S.ERR_ARG),                          # too many scalars
    ([T(S.LOAD, 0)], -1, 0, S.ERR_ARG),
])
def test_program_rejected(prog, nops, nsc, code):
    with pytest.raises(S.SaltError) as e:
        S.salt_program_check(prog, nops, nsc)
    assert e.value.status == code
    assert S.lib().salt_last_error()


def test_program_accepted_and_measured():
    assert S.salt_program_check(FIG1, 3, 0) == (3, 3)
    assert S.salt_program_check([T(S.LOAD, 0)] * 8 + [T(S.ADD)] * 7, 1, 0) == (8, 1)
    assert S.salt_program_check([T(S.SCALAR, 2)], 0, 3) == (1, 0)
    # 62 tokens, left-deep: never more than 2 values on the stack
    left_deep = [T(S.LOAD, 0), T(S.LOAD, 1)] + [T(S.ADD), T(S.LOAD, 0)] * 29 + [T(S.ADD)]
    assert S.salt_program_check(left_deep, 2, 0) == (2, 2)


def test_catalogue_is_canonical_and_routes_to_itself():
    cat = S.salt_catalogue()
    names = [n for n, _ in cat]
    assert names[:3] == ["copy", "scale", "fig1"]
    progs = dict(cat)
    assert progs["fig1"] == FIG1
    assert progs["axpy"] == [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL), T(S.LOAD, 1), T(S.ADD)]
    assert progs["tree5"] == [T(S.LOAD, 0), T(S.LOAD, 1), T(S.MUL), T(S.LOAD, 2), T(S.LOAD, 3), T(S.MUL),
                              T(S.ADD), T(S.LOAD, 4), T(S.SUB)]
    for i, (name, prog) in enumerate(cat):
        nops = 1 + max([t >> 8 for t in prog if t & 0xFF == S.LOAD], default=-1)
        nsc = 1 + max([t >> 8 for t in prog if t & 0xFF == S.SCALAR], default=-1)
        assert S.salt_program_route(prog, nops, nsc) == i, name


def test_routing_ignores_operand_numbering():
    # d = c + (a - b): the Fig. 1 shape with operands renumbered
    prog = [T(S.LOAD, 2), T(S.LOAD, 0), T(S.LOAD, 1), T(S.SUB), T(S.ADD)]
    assert S.salt_program_route(prog, 3, 0) == S.salt_program_route(FIG1, 3, 0)
    # extra unused operands and scalars do not matter either
    assert S.salt_program_route(prog, 8, 8) == S.salt_program_route(FIG1, 3, 0)
    # a different shape goes to the interpreter
    assert S.salt_program_route([T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD), T(S.LOAD, 2), T(S.SUB)], 3, 0) == -1
    # the same operand twice is a different tree from two operands
    assert S.salt_program_route([T(S.LOAD, 0), T(S.LOAD, 0), T(S.LOAD, 0), T(S.SUB), T(S.ADD)], 1, 0) == -1


# ---------------------------------------------------------------------------
# entry points reject bad arguments before any launch
# ---------------------------------------------------------------------------

def _eval(L, prog, ops, scalars, out, n, dtype, cfg=None):
    parr = (ctypes.c_uint32 * max(1, len(prog)))(*prog)
    oa = (ctypes.c_void_p * max(1, len(ops)))(*ops)
    sa = (ctypes.c_double * max(1, len(scalars)))(*scalars)
    if cfg is None:
        return L.salt_eval(parr, len(prog), oa, len(ops), sa, len(scalars), out, n, dtype, None)
    return L.salt_eval_ex(parr, len(prog), oa, len(ops), sa, len(scalars), out, n, dtype, None,
                          ctypes.byref(S.LaunchConfig(*cfg)))


def test_eval_argument_errors(L):
    A, B, C, OUT = 0x10000, 0x20000, 0x30000, 0x40000
    assert _eval(L, FIG1, [A, B, C], [], OUT, -1, S.F64) == S.ERR_ARG
    assert _eval(L, FIG1, [A, B, C], [], OUT, 10, 7) == S.ERR_ARG
    assert _eval(L, FIG1, [A, B, C], [], None, 10, S.F64) == S.ERR_ARG
    assert _eval(L, FIG1, [A, None, C], [], OUT, 10, S.F64) == S.ERR_ARG
    assert b"operand 1" in L.salt_last_error()
    # output partially overlapping an operand
    assert _eval(L, FIG1, [A, B, C], [], A + 8, 10, S.F64) == S.ERR_ARG
    assert b"overlap" in L.salt_last_error()
    assert _eval(L, FIG1, [A, B, C], [], B - 4, 2, S.F32) == S.ERR_ARG
    # bad program is reported as such even with good pointers
    assert _eval(L, FIG1[:-1], [A, B, C], [], OUT, 10, S.F64) == S.ERR_PROGRAM
    # unroll values outside the compiled set
    assert _eval(L, FIG1, [A, B, C], [], OUT, 10, S.F64, cfg=(3, -1, -1)) == S.ERR_ARG
    assert _eval(L, FIG1, [A, B, C], [], OUT, 10, S.F64, cfg=(0, 2, -1)) == S.ERR_ARG
    # n == 0 is a valid no-op: nothing is launched, even with null pointers
    assert _eval(L, FIG1, [None, None, None], [], None, 0, S.F64) == S.OK
    # scalar array missing
    parr = (ctypes.c_uint32 * 3)(T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL))
    oa = (ctypes.c_void_p * 1)(A)
    assert L.salt_eval(parr, 3, oa, 1, None, 1, OUT, 10, S.F64, None) == S.ERR_ARG


def test_axpy_argument_errors(L):
    assert L.salt_axpy(-1, 2.0, 0x1000, 0x2000, S.F64, None) == S.ERR_ARG
    assert L.salt_axpy(10, 2.0, 0x1000, 0x1008, S.F64, None) == S.ERR_ARG   # x overlaps y
    assert L.salt_axpy(10, 2.0, None, 0x2000, S.F32, None) == S.ERR_ARG
    assert L.salt_axpy(0, 2.0, None, None, S.F32, None) == S.OK


def test_reduce_workspace_size(L):
    for d in (S.F64, S.F32, S.BF16, S.F16):
        T_ = S.salt_reduce_tile_elems(d)
        assert T_ * S.ELEM_BYTES[d] == 64 * 1024  # 64 KiB per operand per tile
        assert S.salt_reduce_workspace_bytes(0, d) == 0
        assert S.salt_reduce_workspace_bytes(-5, d) == 0
        assert S.salt_reduce_workspace_bytes(1, d) == 8
        assert S.salt_reduce_workspace_bytes(T_, d) == 8
        assert S.salt_reduce_workspace_bytes(T_ + 1, d) == 16
        assert S.salt_reduce_workspace_bytes(1 << 28, d) == 8 * ((1 << 28) // T_)


def test_reduce_argument_errors(L):
    X, Y, R, W = 0x100000, 0x200000, 0x300000, 0x400000
    n = 100000
    need = S.salt_reduce_workspace_bytes(n, S.F64)
    assert L.salt_dot(-1, X, Y, R, W, need, S.F64, None) == S.ERR_ARG
    assert L.salt_dot(n, X, Y, None, W, need, S.F64, None) == S.ERR_ARG
    assert L.salt_dot(n, X, None, R, W, need, S.F64, None) == S.ERR_ARG
    assert L.salt_dot(n, X, Y, R, None, need, S.F64, None) == S.ERR_WORKSPACE
    assert L.salt_dot(n, X, Y, R, W, need - 8, S.F64, None) == S.ERR_WORKSPACE
    assert L.salt_dot(n, X, Y, R, W + 4, need, S.F64, None) == S.ERR_WORKSPACE
    assert L.salt_dot(n, X, Y, R, X + 64, need, S.F64, None) == S.ERR_WORKSPACE   # overlaps x
    assert L.salt_nrm2(n, X, R, W, need - 8, S.F64, None) == S.ERR_WORKSPACE
    assert L.salt_nrm2(n, X, R, W, need, 11, None) == S.ERR_ARG
    cfg = ctypes.byref(S.LaunchConfig(3, -1, -1))
    assert L.salt_dot_ex(n, X, Y, R, W, need, S.F64, None, cfg) == S.ERR_ARG


def test_tuning_table(tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("# kind route dtype log2n unroll nt blocks\n"
                 "eval 2 0 20 2 0 0\n"
                 "eval 2 0 28 8 1 1024\n"
                 "dot -1 1 26 16 1 2048\n")
    S.salt_tuning_load(str(p))
    try:
        assert S.salt_tuning_lookup(0, 2, S.F64, 1 << 20) == (2, 0, 0)
        assert S.salt_tuning_lookup(0, 2, S.F64, 1 << 27) == (8, 1, 1024)   # nearest bucket
        assert S.salt_tuning_lookup(1, -1, S.F32, 1 << 10) == (16, 1, 2048)
        # no row: the built-in default
        assert S.salt_tuning_lookup(0, 4, S.F32, 1 << 10)[2] == 0
        bad = tmp_path / "bad.txt"
        bad.write_text("eval 2 0\n")
        with pytest.raises(S.SaltError):
            S.salt_tuning_load(str(bad))
        with pytest.raises(S.SaltError):
            S.salt_tuning_load(str(tmp_path / "missing.txt"))
        # a failed load leaves the previous table in place
        assert S.salt_tuning_lookup(0, 2, S.F64, 1 << 20) == (2, 0, 0)
    finally:
        try:
            S.salt_tuning_load(None)   # back to the packaged table
        except S.SaltError:
            empty = tmp_path / "empty.txt"
            empty.write_text("")
            S.salt_tuning_load(str(empty))


def test_tuning_lookup_is_the_nearest_row_of_the_packaged_table():
    """Every (kind, route, dtype) of the packaged table at every log2 size:
    the library's lookup returns the row nearest in log2 n, the first in
    file order among equally near rows (a scan of the file, written out
    here)."""
    path = os.path.join(ROOT, "paper_1109_1264_amd", "salt_tuning.txt")
    kinds = {"eval": 0, "dot": 1, "nrm2": 2, "batch": 3}
    rows = []
    for line in open(path):
        f = line.split("#")[0].split()
        if f:
            rows.append((kinds[f[0]], int(f[1]), int(f[2]), int(f[3]), (int(f[4]), int(f[5]), int(f[6]))))
    S.salt_tuning_load(None)
    keys = sorted({r[:3] for r in rows})
    assert len(keys) > 50
    for kind, route, dt in keys:
        mine = [r for r in rows if r[:3] == (kind, route, dt)]
        for l in range(0, 60):
            best = min(mine, key=lambda r: abs(r[3] - l))      # min keeps the first of equals
            assert S.salt_tuning_lookup(kind, route, dt, 1 << l) == best[4], (kind, route, dt, l)
        # sizes between powers of two use the floor of log2 n
        assert S.salt_tuning_lookup(kind, route, dt, 3 << 20) == S.salt_tuning_lookup(kind, route, dt, 1 << 21)


def test_reduce_expr_argument_errors(L):
    X, Y, R, W = 0x100000, 0x200000, 0x300000, 0x400000
    n = 100000
    need = S.salt_reduce_workspace_bytes(n, S.F64)
    px = (ctypes.c_uint32 * 1)(T(S.LOAD, 0))
    py = (ctypes.c_uint32 * 1)(T(S.LOAD, 1))
    bad = (ctypes.c_uint32 * 1)(T(S.ADD))
    ops = (ctypes.c_void_p * 2)(X, Y)
    ops_null = (ctypes.c_void_p * 2)(X, None)
    sc = (ctypes.c_double * 1)(1.0)
    f = L.salt_dot_expr
    assert f(bad, 1, py, 1, ops, 2, sc, 0, n, R, W, need, S.F64, None) == S.ERR_PROGRAM
    assert b"first program" in L.salt_last_error()
    assert f(px, 1, bad, 1, ops, 2, sc, 0, n, R, W, need, S.F64, None) == S.ERR_PROGRAM
    assert f(px, 1, py, 1, ops_null, 2, sc, 0, n, R, W, need, S.F64, None) == S.ERR_ARG
    assert f(px, 1, py, 1, ops, 2, sc, 0, n, None, W, need, S.F64, None) == S.ERR_ARG
    assert f(px, 1, py, 1, ops, 2, sc, 0, n, R, W, need - 8, S.F64, None) == S.ERR_WORKSPACE
    assert f(px, 1, py, 1, ops, 2, sc, 0, -1, R, W, need, S.F64, None) == S.ERR_ARG
    assert L.salt_nrm2_expr(px, 1, ops, 2, sc, 0, n, R, X + 8, need, S.F64, None) == S.ERR_WORKSPACE
    deep = (ctypes.c_uint32 * 15)(*([T(S.LOAD, 0)] * 8 + [T(S.SUB)] * 7))
    assert f(deep, 15, deep, 15, ops, 2, sc, 0, n, R, W, need, S.F64, None) == S.ERR_UNSUPPORTED


def test_blas1_strided_argument_errors(L):
    """Strided BLAS level-1: rejected arguments, and the calls that do nothing
    (n = 0, or inc <= 0 for scal) return OK without touching the device."""
    X, Y, R, W = 0x1000000, 0x2000000, 0x3000000, 0x4000000
    F64, F32 = S.F64, S.F32
    # scal
    assert L.salt_scal(-1, 2.0, X, 1, F64, None) == S.ERR_ARG
    assert L.salt_scal(5, 2.0, None, 2, F64, None) == S.ERR_ARG
    assert L.salt_scal(5, 2.0, X, 2, 9, None) == S.ERR_ARG
    assert L.salt_scal(1 << 40, 2.0, X, 1 << 20, F64, None) == S.ERR_ARG      # span past 2^59
    assert L.salt_scal(5, 2.0, X, 0, F64, None) == S.OK                       # reference BLAS: no-op
    assert L.salt_scal(5, 2.0, X, -3, F64, None) == S.OK
    assert L.salt_scal(0, 2.0, None, 1, F64, None) == S.OK
    # copy / axpy: an output increment of 0 with n > 1 is rejected
    assert L.salt_copy(3, X, 1, Y, 0, F32, None) == S.ERR_ARG
    assert L.salt_copy(3, None, 2, Y, 1, F32, None) == S.ERR_ARG
    assert L.salt_copy(-2, X, 1, Y, 1, F32, None) == S.ERR_ARG
    assert L.salt_copy(0, None, 1, None, 1, F32, None) == S.OK
    assert L.salt_axpy_strided(3, 1.0, X, 0, Y, 0, F64, None) == S.ERR_ARG
    assert L.salt_axpy_strided(3, 1.0, X, 2, None, 1, F64, None) == S.ERR_ARG
    assert L.salt_axpy_strided(1 << 50, 1.0, X, 1, Y, -(1 << 12), F64, None) == S.ERR_ARG
    # strided reductions: result, workspace size, alignment and overlap
    n, inc = 100000, 3
    need = S.salt_reduce_workspace_bytes(n, F64)
    assert L.salt_dot_strided(n, X, inc, Y, 2, None, W, need, F64, None) == S.ERR_ARG
    assert L.salt_dot_strided(n, X, inc, Y, 2, R, None, need, F64, None) == S.ERR_WORKSPACE
    assert L.salt_dot_strided(n, X, inc, Y, 2, R, W, need - 8, F64, None) == S.ERR_WORKSPACE
    assert L.salt_dot_strided(n, X, -inc, Y, 2, R, W + 4, need, F64, None) == S.ERR_WORKSPACE
    # the span of x with |inc| = 3 reaches X + 8*(1 + 3(n-1)); a workspace inside it
    assert L.salt_dot_strided(n, X, -inc, Y, 2, R, X + 8 * 3 * (n - 10), need, F64, None) == S.ERR_WORKSPACE
    assert L.salt_dot_strided(n, None, inc, Y, 2, R, W, need, F64, None) == S.ERR_ARG
    assert L.salt_nrm2_strided(n, X, inc, R, W, need - 8, F64, None) == S.ERR_WORKSPACE
    assert L.salt_asum(n, X, inc, R, W + 4, need, F64, None) == S.ERR_WORKSPACE
    assert L.salt_asum(-1, X, inc, R, W, need, F64, None) == S.ERR_ARG
    # iamax: int64 result, 8-byte aligned; workspace as the reductions
    assert L.salt_iamax(n, X, inc, None, W, need, F64, None) == S.ERR_ARG
    assert L.salt_iamax(n, X, inc, R + 4, W, need, F64, None) == S.ERR_ARG
    assert L.salt_iamax(n, X, inc, R, W, need - 8, F64, None) == S.ERR_WORKSPACE
    assert L.salt_iamax(n, None, inc, R, W, need, F64, None) == S.ERR_ARG


def test_sharded_reduction_argument_errors(L):
    X, Y, P, R = 0x1000000, 0x2000000, 0x3000000, 0x4000000
    n = 100000
    assert L.salt_reduce_partials(3, n, X, Y, P, S.F64, None) == S.ERR_ARG           # mode
    assert L.salt_reduce_partials(0, -1, X, Y, P, S.F64, None) == S.ERR_ARG
    assert L.salt_reduce_partials(0, n, X, None, P, S.F64, None) == S.ERR_ARG        # dot needs y
    assert L.salt_reduce_partials(1, n, X, None, None, S.F64, None) == S.ERR_ARG     # no partials
    assert L.salt_reduce_partials(1, n, X, None, P + 4, S.F64, None) == S.ERR_ARG    # misaligned
    assert L.salt_reduce_partials(1, n, X, None, X + 64, S.F64, None) == S.ERR_ARG   # overlaps x
    assert L.salt_reduce_partials(0, n, X, Y, P, 7, None) == S.ERR_ARG               # dtype
    assert L.salt_reduce_partials(2, 0, None, None, None, S.F32, None) == S.OK       # empty shard: nothing to do
    assert L.salt_reduce_combine(-1, P, 4, R, S.F64, None) == S.ERR_ARG
    assert L.salt_reduce_combine(0, P, -1, R, S.F64, None) == S.ERR_ARG
    assert L.salt_reduce_combine(0, P, 4, None, S.F64, None) == S.ERR_ARG
    assert L.salt_reduce_combine(0, None, 4, R, S.F64, None) == S.ERR_ARG
    assert L.salt_reduce_combine(0, P + 2, 4, R, S.F64, None) == S.ERR_ARG


def test_stream_reference_argument_errors(L):
    """The stream reference rejects bad shapes before any launch (fake
    16-byte aligned addresses are never dereferenced)."""
    fake = (ctypes.c_void_p * 6)(*([1 << 40] * 6))
    out = ctypes.c_void_p(1 << 41)
    assert L.salt_stream_reference(0, 1, fake, out, 64, None) == S.ERR_ARG      # no input
    assert L.salt_stream_reference(7, 1, fake, out, 64, None) == S.ERR_ARG      # too many inputs
    assert L.salt_stream_reference(2, 2, fake, out, 64, None) == S.ERR_ARG      # two outputs
    assert L.salt_stream_reference(2, 1, fake, out, 40, None) == S.ERR_ARG      # not whole chunks
    assert L.salt_stream_reference(2, 1, fake, out, -16, None) == S.ERR_ARG
    assert L.salt_stream_reference(2, 1, fake, None, 64, None) == S.ERR_ARG     # output missing
    odd = (ctypes.c_void_p * 2)((1 << 40) + 8, 1 << 40)
    assert L.salt_stream_reference(2, 1, odd, out, 64, None) == S.ERR_ARG       # misaligned input
    assert L.salt_stream_reference(2, 1, fake, out, 0, None) == S.OK           # nothing to do


def test_reduce_expr_route_matches_the_pair_catalogue():
    """Expression reductions that match a catalogue pair under canonical
    numbering (operands and scalars by first use, P then Q; a dot's programs
    in either order) route to its ahead-of-time kernel; anything else to the
    interpreter (-1). Host only."""
    L0, L1, L2, L3 = T(S.LOAD, 0), T(S.LOAD, 1), T(S.LOAD, 2), T(S.LOAD, 3)
    ADD, SUB, MUL = T(S.ADD), T(S.SUB), T(S.MUL)
    r = S.salt_reduce_expr_route
    assert r([L0, L1, ADD], [L0, L1, SUB], 2, 0) == 0            # dot(a + b, a - b)
    assert r([L2, L3, ADD], [L2, L3, SUB], 4, 0) == 0            # other operand numbers
    assert r([L0, L1, SUB], [L0, L1, ADD], 2, 0) == 0            # programs exchanged
    assert r([L1, L0, ADD], [L0, L1, SUB], 2, 0) == -1           # b + a: not the same tokens
    assert r([L0, L1, ADD], [L1, L0, SUB], 2, 0) == -1           # a + b with b - a
    assert r([L0, L1, SUB], None, 2, 0) == 1                     # nrm2(a - b)
    assert r([L1, L0, SUB], None, 2, 0) == 1                     # nrm2(b - a): renumbered
    assert r([L0, L1, ADD], None, 2, 0) == -1
    assert r([L0, L1, SUB], [L0, L1, SUB], 2, 0) == -1           # a dot, not a norm
    assert r([T(S.SCALAR, 0), L0, MUL, L1, ADD], None, 2, 1) == 2   # nrm2(alpha*a + b)
    assert r([T(S.SCALAR, 2), L3, MUL, L0, ADD], None, 4, 3) == 2   # other numbers
    assert r([L0, T(S.SCALAR, 0), MUL, L1, ADD], None, 2, 1) == -1  # a*alpha: other tokens
    assert r([T(S.SCALAR, 0), L0, MUL, L0, ADD], None, 2, 1) == -1  # one operand twice
    with pytest.raises(S.SaltError):
        r([L0, L1, ADD], [L0, L2, SUB], 2, 0)                     # operand out of range


def test_eval_chunking_policy():
    """Large calls of trees reading three or more operands run as launches of
    128 MiB per operand (the last takes the remainder); others as one."""
    c64 = (128 << 20) // 8
    assert S.salt_eval_chunking(5, 1 << 28, S.F64) == (c64, 16)
    assert S.salt_eval_chunking(5, 2 * c64 - 1, S.F64) == (2 * c64 - 1, 1)   # below two chunks
    assert S.salt_eval_chunking(3, 2 * c64, S.F64) == (c64, 2)
    assert S.salt_eval_chunking(3, 3 * c64 - 1, S.F64) == (c64, 2)           # remainder in the last
    assert S.salt_eval_chunking(2, 1 << 28, S.F64) == (1 << 28, 1)           # axpy-like: one launch
    assert S.salt_eval_chunking(1, 1 << 28, S.F64) == (1 << 28, 1)
    assert S.salt_eval_chunking(5, 1 << 28, S.BF16) == ((128 << 20) // 2, 4)
    assert S.salt_eval_chunking(6, 0, S.F32) == (0, 0)
    with pytest.raises(S.SaltError):
        S.salt_eval_chunking(9, 10, S.F32)
    with pytest.raises(S.SaltError):
        S.salt_eval_chunking(3, -1, S.F32)
