"""Pins of the CPU oracle against things other than itself.

Each check is a function of the oracle module so that the mutation test
(``test_oracle_mutants.py``) can run the same checks against deliberately
broken builds of the oracle and see them fail.

Pins used (none retypes the oracle's own loops):
- the paper's Fig. 1 tree on hand-worked dyadic rows (``golden/``);
- the same trees written as ordinary Python / numpy expressions (IEEE
  binary64 / binary32 arithmetic of the interpreter and of numpy);
- random postfix programs turned into infix source text and evaluated by
  Python itself;
- closed forms (a_i = i, b_i = 2i, c_i = i; dot = n(n-1)(2n-1)/3; nrm2 of
  ones and of 0..n-1);
- exact rational arithmetic (``fractions.Fraction``) and ``math.fsum`` for the
  reductions, within the Dot2 error bound of Ogita, Rump and Oishi (2005);
- torch / numpy conversions to bfloat16 / binary16 and hand-worked rounding
  cases for the 16-bit storage formats;
- numpy slicing for BLAS strided vectors (x[::inc], reversed for inc < 0),
  numpy ``argmax`` (first occurrence) and hand-worked NaN / tie cases for
  iamax, and ``math.fsum`` for asum;
- for the replay of the library's summation order: hand-worked inputs whose
  result depends on that order, exact integer sums and the Dot2 bound.
"""
from __future__ import annotations

import math
import os
import random
import struct
from fractions import Fraction

import numpy as np
import pytest

from paper_1109_1264_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LOAD, SCALAR, ADD, SUB, MUL = 1, 2, 3, 4, 5
U64 = 2.0 ** -53


def tok(op, arg=0):
    return (arg << 8) | op


FIG1 = [tok(LOAD, 0), tok(LOAD, 1), tok(LOAD, 2), tok(SUB), tok(ADD)]          # a + (b - c)
TREE5 = [tok(LOAD, 0), tok(LOAD, 1), tok(MUL), tok(LOAD, 2), tok(LOAD, 3), tok(MUL),
         tok(ADD), tok(LOAD, 4), tok(SUB)]                                   # a*b + c*e - f
AXPY = [tok(SCALAR, 0), tok(LOAD, 0), tok(MUL), tok(LOAD, 1), tok(ADD)]       # alpha*x + y


def bits64(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


def bits32(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def postfix_to_infix(prog):
    """Source text of the expression a postfix program denotes
    (pop r, pop l, push (l op r))."""
    st = []
    sym = {ADD: "+", SUB: "-", MUL: "*"}
    for t in prog:
        op, arg = t & 0xFF, t >> 8
        if op == LOAD:
            st.append("x%d" % arg)
        elif op == SCALAR:
            st.append("s%d" % arg)
        else:
            r = st.pop()
            l = st.pop()
            st.append("(%s %s %s)" % (l, sym[op], r))
    assert len(st) == 1
    return st[0]


def random_program(rng, n_ops, n_sc, max_leaves=7):
    """A random tree over the given operands and scalars, as postfix."""
    def build(leaves):
        if leaves == 1:
            if n_sc and rng.random() < 0.25:
                return [tok(SCALAR, rng.randrange(n_sc))]
            return [tok(LOAD, rng.randrange(n_ops))]
        k = rng.randrange(1, leaves)
        return build(k) + build(leaves - k) + [tok(rng.choice([ADD, SUB, MUL]))]
    return build(rng.randrange(1, max_leaves + 1))


# --------------------------------------------------------------------------
# element-wise: binary64
# --------------------------------------------------------------------------

def check_fig1_golden(o):
    rows = [list(map(float, l.split())) for l in open(os.path.join(GOLDEN, "fig1_tree_dyadic.txt"))
            if l.strip() and not l.startswith("#")]
    a, b, c, d = (np.array(col) for col in zip(*rows))
    for dt in ("f64", "f32"):
        got = o.eval_program(FIG1, [a, b, c], [], dt)
        assert np.array_equal(got, d.astype(got.dtype)), (dt, got, d)


def check_python_float_trees_f64(o):
    a, b, c, e, f = workloads.uniform(301, "f64", 11, 5)
    got = o.eval_program(FIG1, [a, b, c], [], "f64")
    want = [float(x) + (float(y) - float(z)) for x, y, z in zip(a, b, c)]
    assert np.array_equal(bits64(got), bits64(want))
    got = o.eval_program(TREE5, [a, b, c, e, f], [], "f64")
    want = [float(p) * float(q) + float(r) * float(s) - float(t) for p, q, r, s, t in zip(a, b, c, e, f)]
    assert np.array_equal(bits64(got), bits64(want))
    al = workloads.alpha(11)
    got = o.eval_program(AXPY, [a, b], [al], "f64")
    want = [al * float(x) + float(y) for x, y in zip(a, b)]
    assert np.array_equal(bits64(got), bits64(want))


def check_random_programs(o, dtype, count=150):
    rng = random.Random(1234 + len(dtype))
    n = 67
    np_t = np.float64 if dtype == "f64" else np.float32
    for _ in range(count):
        n_ops, n_sc = rng.randint(1, 8), rng.randint(0, 8)
        prog = random_program(rng, n_ops, n_sc)
        ops = workloads.uniform(n, dtype, rng.randrange(1 << 30), n_ops)
        sc = [rng.uniform(-3, 3) for _ in range(n_sc)]
        env = {"x%d" % k: ops[k] for k in range(n_ops)}
        env.update({"s%d" % j: np_t(sc[j]) for j in range(n_sc)})
        src = postfix_to_infix(prog)
        want = np.broadcast_to(np.asarray(eval(src, {}, env), dtype=np_t), (n,))
        got = o.eval_program(prog, ops, sc, dtype, n=n)
        assert got.dtype == np_t
        assert np.array_equal(got.view(np.uint64 if dtype == "f64" else np.uint32),
                              np.ascontiguousarray(want).view(np.uint64 if dtype == "f64" else np.uint32)), src


def check_closed_form(o):
    n = 1 << 16
    i = np.arange(n, dtype=np.float64)
    got = o.eval_program(FIG1, [i, 2 * i, i], [], "f64")
    assert np.array_equal(got, 2 * i)
    m = 1 << 23  # 2i <= 2^24 stays exact in binary32
    i32 = np.arange(0, m, 997, dtype=np.float32)
    got = o.eval_program(FIG1, [i32, 2 * i32, i32], [], "f32")
    assert np.array_equal(got, 2 * i32)


def check_invariants(o, dtype):
    a, b = workloads.uniform(513, dtype, 99, 2)
    zero = o.eval_program([tok(LOAD, 0), tok(LOAD, 0), tok(SUB)], [a], [], dtype)
    assert not np.any(zero.view(np.uint64 if dtype == "f64" else np.uint32))  # all +0
    for op in (ADD, MUL):
        ab = o.eval_program([tok(LOAD, 0), tok(LOAD, 1), tok(op)], [a, b], [], dtype)
        ba = o.eval_program([tok(LOAD, 1), tok(LOAD, 0), tok(op)], [a, b], [], dtype)
        assert np.array_equal(ab.view(np.uint8), ba.view(np.uint8))
    one = o.eval_program([tok(LOAD, 0), tok(SCALAR, 0), tok(MUL)], [a], [1.0], dtype)
    assert np.array_equal(one.view(np.uint8), a.view(np.uint8))
    plus0 = o.eval_program([tok(LOAD, 0), tok(SCALAR, 0), tok(ADD)], [a], [0.0], dtype)
    assert np.array_equal(plus0.view(np.uint8), a.view(np.uint8))


def check_f32_numpy_trees(o):
    a, b, c, e, f = workloads.uniform(1001, "f32", 5, 5)
    assert np.array_equal(bits32(o.eval_program(FIG1, [a, b, c], [], "f32")), bits32(a + (b - c)))
    assert np.array_equal(bits32(o.eval_program(TREE5, [a, b, c, e, f], [], "f32")),
                          bits32(a * b + c * e - f))
    # scalars are rounded once to binary32
    al = 1.0 / 3.0
    got = o.eval_program(AXPY, [a, b], [al], "f32")
    assert np.array_equal(bits32(got), bits32(np.float32(al) * a + b))


def check_subnormals(o):
    # binary64 subnormals stay (no flush to zero)
    tiny = np.array([5e-324, 2.5e-320, -1e-310, 2.2250738585072014e-308], dtype=np.float64)
    got = o.eval_program([tok(LOAD, 0), tok(SCALAR, 0), tok(MUL)], [tiny], [0.5], "f64")
    want = [float(t) * 0.5 for t in tiny]
    assert np.array_equal(bits64(got), bits64(want))
    t32 = np.array([1e-45, 3e-42, -1.1754942e-38, 1.17549435e-38], dtype=np.float32)
    got = o.eval_program([tok(LOAD, 0), tok(LOAD, 0), tok(ADD)], [t32], [], "f32")
    assert np.array_equal(bits32(got), bits32(t32 + t32))
    assert np.all(got[:3] != 0)


# --------------------------------------------------------------------------
# 16-bit storage
# --------------------------------------------------------------------------

def check_rounding_golden(o):
    for line in open(os.path.join(GOLDEN, "rounding_16bit.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        fmt, fbits, hbits = line.split()[:3]
        f = struct.unpack("<f", struct.pack("<I", int(fbits, 16)))[0]
        got = int(o.narrow([f], fmt)[0])
        assert got == int(hbits, 16), (line, hex(got))


def check_conversions_vs_libraries(o):
    import torch

    allh = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    # widening: every 16-bit pattern (NaNs compared as NaN)
    w_bf = o.widen(allh, "bf16")
    ref_bf = torch.from_numpy(allh.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    w_h = o.widen(allh, "f16")
    ref_h = allh.view(np.float16).astype(np.float64)
    for got, ref in ((w_bf, ref_bf), (w_h, ref_h)):
        nan = np.isnan(ref)
        assert np.array_equal(np.isnan(got), nan)
        assert np.array_equal(bits64(got[~nan]), bits64(ref[~nan]))
    # narrowing: random binary32 patterns across all exponents, plus ties
    rng = np.random.Generator(np.random.PCG64(77))
    pats = rng.integers(0, 1 << 32, 400000, dtype=np.uint64).astype(np.uint32)
    ties = (rng.integers(0, 1 << 16, 50000, dtype=np.uint64).astype(np.uint32) << 16) | 0x8000
    ties16 = (rng.integers(0, 1 << 19, 50000, dtype=np.uint64).astype(np.uint32) << 13) | 0x1000
    f = np.concatenate([pats, ties, ties16]).view(np.float32)
    f = f[~np.isnan(f)]
    got = o.narrow(f, "bf16")
    ref = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, ref)
    got = o.narrow(f, "f16")
    with np.errstate(over="ignore"):
        ref = f.astype(np.float16).view(np.uint16)
    assert np.array_equal(got, ref)


def check_h16_eval_composition(o, dtype):
    """16-bit storage eval = widen, binary32 ops, one narrowing (torch / numpy)."""
    import torch

    a, b, c, e, f = workloads.uniform(777, dtype, 21, 5)
    tt = torch.bfloat16 if dtype == "bf16" else torch.float16

    def wid(h):
        return torch.from_numpy(h.view(np.int16)).view(tt).to(torch.float32).numpy()

    def nar(x):
        return torch.from_numpy(np.ascontiguousarray(x)).to(tt).view(torch.int16).numpy().view(np.uint16)

    A, B, C, E, F = map(wid, (a, b, c, e, f))
    assert np.array_equal(o.eval_program(FIG1, [a, b, c], [], dtype), nar(A + (B - C)))
    assert np.array_equal(o.eval_program(TREE5, [a, b, c, e, f], [], dtype), nar(A * B + C * E - F))
    al = 1.2345678901
    assert np.array_equal(o.eval_program(AXPY, [a, b], [al], dtype), nar(np.float32(al) * A + B))


# --------------------------------------------------------------------------
# axpy
# --------------------------------------------------------------------------

def check_axpy(o):
    x, y = workloads.uniform(999, "f64", 3, 2)
    al = workloads.alpha(3)
    got = o.axpy(al, x, y, "f64")
    assert np.array_equal(bits64(got), bits64([al * float(p) + float(q) for p, q in zip(x, y)]))
    x32, y32 = workloads.uniform(999, "f32", 3, 2)
    got = o.axpy(al, x32, y32, "f32")
    assert np.array_equal(bits32(got), bits32(np.float32(al) * x32 + y32))
    # alpha = 2 on small integers is exact: y = 2x + y
    i = np.arange(-500, 500, dtype=np.float64)
    assert np.array_equal(o.axpy(2.0, i, 3 * i, "f64"), 5 * i)
    assert np.array_equal(o.axpy(0.5, i.astype(np.float32), i.astype(np.float32), "f32"),
                          (1.5 * i).astype(np.float32))


# --------------------------------------------------------------------------
# reductions
# --------------------------------------------------------------------------

def dot2_bound(n, exact_abs, sum_abs):
    """Ogita-Rump-Oishi (2005) Prop. 5.5 bound for Dot2 in binary64."""
    g = n * U64 / (1 - n * U64)
    return U64 * exact_abs + g * g * sum_abs + 1e-300


def check_dot_closed_form(o):
    for n in (0, 1, 2, 3, 10, 1000, 1 << 17):
        i = np.arange(n, dtype=np.float64)
        r, _ = o.dot2(i, 2 * i)
        assert r == n * (n - 1) * (2 * n - 1) // 3, n
    # beyond 2^53 the value is no longer an integer in binary64: within Dot2's bound
    n = 1 << 20
    i = np.arange(n, dtype=np.float64)
    r, s = o.dot2(i, 2 * i)
    exact = Fraction(n * (n - 1) * (2 * n - 1), 3)
    assert abs(Fraction(r) - exact) <= Fraction(dot2_bound(n, float(exact), s))


def check_dot_fraction_bruteforce(o):
    rng = np.random.Generator(np.random.PCG64(2024))
    for trial in range(300):
        n = int(rng.integers(0, 17))
        x = rng.standard_normal(n) * 10.0 ** rng.integers(-5, 5, n)
        y = rng.standard_normal(n) * 10.0 ** rng.integers(-5, 5, n)
        if trial % 3 == 0 and n >= 2:   # cancellation: y ~ -x on half the terms
            y[: n // 2] = -x[: n // 2] * (1 + 1e-12)
        exact = sum((Fraction(float(p)) * Fraction(float(q)) for p, q in zip(x, y)), Fraction(0))
        r, s = o.dot2(x, y)
        assert abs(Fraction(r) - exact) <= Fraction(dot2_bound(n, abs(float(exact)), s)), (n, r, float(exact))


def check_dot_fsum(o):
    """binary32 inputs: every product is exact in binary64, so math.fsum of
    the products is the correctly rounded exact dot product."""
    x64, y64 = workloads.ill_conditioned(200000, 31)
    x = x64.astype(np.float32).astype(np.float64)
    y = y64.astype(np.float32).astype(np.float64)
    exact = math.fsum((x * y).tolist())
    r, s = o.dot2(x, y)
    assert abs(r - exact) <= dot2_bound(len(x), abs(exact), s)
    # and the plain binary64 loop is visibly worse than Dot2 on this data
    assert abs(o.naive_dot(x, y) - exact) >= abs(r - exact)


def check_nrm2(o):
    for k in range(0, 11):
        n = 4 ** k
        assert o.nrm2(np.ones(n)) == 2.0 ** k
    assert o.nrm2(np.zeros(0)) == 0.0
    for n in (2, 7, 100, 4097):
        i = np.arange(n, dtype=np.float64)
        exact = Fraction((n - 1) * n * (2 * n - 1), 6)
        r = o.nrm2(i)
        # r is sqrt of a value within Dot2's bound, plus one rounding of sqrt
        assert abs(r * r - float(exact)) <= 4 * U64 * float(exact), n
    x = np.array([3.0, 4.0])
    assert o.nrm2(x) == 5.0
    assert o.nrm2(np.array([-2.0])) == 2.0


def check_naive_f32(o):
    x, y = workloads.uniform(300, "f32", 8, 2)
    s = np.float32(0.0)
    for p, q in zip(x, y):
        s = np.float32(s + np.float32(p * q))
    assert o.naive_dot(x, y, "f32") == float(s)


def check_naive_f64(o):
    """The binary64 loop adds the products one by one, in element order, each
    product rounded before its addition. Every value below is worked by hand
    from that definition."""
    big = 2.0 ** 53
    one = np.ones(3)
    # order: 2^53 + 1 rounds (tie) back to 2^53, twice; a pairwise, reversed,
    # compensated or Dot2 sum gives 2^53 + 2
    assert o.naive_dot(np.array([big, 1.0, 1.0]), one) == big
    # precision: 1 + 2^-30 is exact in binary64 and rounds to 1 in binary32
    assert o.naive_dot(np.array([1.0, 2.0 ** -30]), np.ones(2)) == 1.0 + 2.0 ** -30
    # the last element counts
    assert o.naive_dot(np.array([0.0, 0.0, 5.0]), one) == 5.0
    # no contraction: (1 + 2^-27)(1 - 2^-27) = 1 - 2^-54 rounds (tie, to even)
    # to 1, so -1 + 1 = 0; a fused multiply-add would keep -2^-54
    assert o.naive_dot(np.array([1.0, 1.0 + 2.0 ** -27]), np.array([-1.0, 1.0 - 2.0 ** -27])) == 0.0
    # integer data: exact in any order (closed form n(n-1)(2n-1)/3)
    n = 1000
    i = np.arange(n, dtype=np.float64)
    assert o.naive_dot(i, 2 * i) == n * (n - 1) * (2 * n - 1) / 3
    assert o.naive_dot(np.zeros(0), np.zeros(0)) == 0.0


def check_naive_par(o):
    """All-cores form: thread t of T sums elements [t*n/T, (t+1)*n/T) in order
    and the partials are added in thread order; values worked by hand."""
    big = 2.0 ** 53
    # T = 1 is the sequential loop
    x, y = workloads.uniform(5000, "f64", 12, 2)
    assert o.naive_dot_par(x, y, 1) == (o.naive_dot(x, y), 1)
    # n = 4, T = 2: shares [2^53, 1] -> 2^53 and [1, 1] -> 2; total 2^53 + 2
    assert o.naive_dot_par(np.array([big, 1.0, 1.0, 1.0]), np.ones(4), 2) == (big + 2, 2)
    # n = 5, T = 2: shares [0, 2) and [2, 5): 2^53 and 3; 2^53 + 3 ties to
    # 2^53 + 4 (a [0, 3) / [3, 5) split would give 2^53 + 2)
    assert o.naive_dot_par(np.array([big, 1.0, 1.0, 1.0, 1.0]), np.ones(5), 2)[0] == big + 4
    # n = 3, T = 3: partials 2^53, 1, 1 added in thread order give 2^53
    # (in reverse order 2^53 + 2)
    assert o.naive_dot_par(np.array([big, 1.0, 1.0]), np.ones(3), 3)[0] == big
    # integer data: exact for any split
    i = np.arange(3001, dtype=np.float64)
    assert o.naive_dot_par(i, 2 * i, 7) == (3001 * 3000 * 6001 / 3, 7)


def check_eval_threads(o):
    """The element-wise loops on several threads give the one-thread bits
    (each element is computed alone)."""
    prog = [tok(LOAD, 0), tok(LOAD, 1), tok(MUL), tok(LOAD, 2), tok(LOAD, 3), tok(MUL), tok(ADD),
            tok(LOAD, 4), tok(SUB)]
    for dt in ("f64", "f32"):
        ops = workloads.uniform(100003, dt, 21, 5)
        one = o.eval_program(prog, ops, [], dt)
        ax1 = o.axpy(1.375, ops[0], ops[1], dt)
        o.set_threads(5)
        try:
            many = o.eval_program(prog, ops, [], dt)
            ax5 = o.axpy(1.375, ops[0], ops[1], dt)
        finally:
            o.set_threads(1)
        assert np.array_equal(one.view(np.uint8), many.view(np.uint8))
        assert np.array_equal(ax1.view(np.uint8), ax5.view(np.uint8))
        # and the values are the trees' (numpy evaluates the same operations)
        a, b, c, e, f = ops
        assert np.array_equal(many, (a * b + c * e) - f)


# --------------------------------------------------------------------------
# the tests
# --------------------------------------------------------------------------

def check_blas_strides(o):
    """Strided vectors against numpy slicing: inc > 0 takes x[0], x[inc], ...;
    inc < 0 takes the same positions in reverse (reference BLAS); inc = 0
    repeats x[0]."""
    rng = np.random.default_rng(41)
    x = rng.standard_normal(40)
    for n in (0, 1, 5, 13):
        for inc in (1, 2, 3, -1, -2, -3):
            span = o.blas_span(n, inc)
            want = x[:span:abs(inc)] if inc > 0 else x[:span:abs(inc)][::-1]
            got = o.gather(n, x, inc)
            assert got.shape == (n,) and np.array_equal(got, want[:n]), (n, inc)
    assert np.array_equal(o.gather(4, x, 0), np.full(4, x[0]))
    # scatter: the strided slots of y take v, every other element is kept
    y = rng.standard_normal(30)
    v = rng.standard_normal(7)
    for inc in (2, -3, 4):
        want = y.copy()
        sl = slice(0, o.blas_span(7, inc), abs(inc))
        want[sl] = v if inc > 0 else v[::-1]
        assert np.array_equal(o.scatter(7, v, y, inc), want), inc
    # copy between two different strides: byte exact, 16-bit patterns too
    h = rng.integers(0, 1 << 16, 50).astype(np.uint16)
    out = o.copy(6, h, -4, np.zeros(20, np.uint16), 3)
    want = np.zeros(20, np.uint16)
    want[0:16:3] = h[0:21:4][::-1]
    assert np.array_equal(out, want)


def check_scal_axpy_strided(o):
    """scal and strided axpy as numpy expressions on slices (binary64 and
    binary32; numpy does not contract), torch for bfloat16 rounding."""
    import torch

    rng = np.random.default_rng(43)
    x = rng.uniform(-2, 2, 64)
    y = rng.uniform(-2, 2, 64)
    alpha = 0.1  # not representable: binary32 must round it once
    for inc in (1, 3, 5):
        n = 12
        sl = slice(0, o.blas_span(n, inc), abs(inc))
        want = x.copy()
        want[sl] = alpha * x[sl]
        assert np.array_equal(bits64(o.scal(n, alpha, x, inc, "f64")), bits64(want)), inc
        x32 = x.astype(np.float32)
        want32 = x32.copy()
        want32[sl] = np.float32(alpha) * x32[sl]
        assert np.array_equal(bits32(o.scal(n, alpha, x32, inc, "f32")), bits32(want32)), inc
    # inc <= 0 leaves x unchanged (reference BLAS)
    assert np.array_equal(o.scal(5, 3.0, x, -1, "f64"), x)
    # bfloat16: binary32 product, one round-to-nearest-even (torch's conversion)
    hb = o.narrow(rng.uniform(-2, 2, 40).astype(np.float32), "bf16")
    got = o.scal(10, alpha, hb, 4, "bf16")
    wide = torch.from_numpy(o.widen(hb, "bf16").astype(np.float32))
    prod = (wide[0:37:4] * torch.tensor(np.float32(alpha))).to(torch.bfloat16).view(torch.int16).numpy()
    want = hb.copy()
    want[0:37:4] = prod.view(np.uint16)
    assert np.array_equal(got, want)
    # strided axpy, x and y with different increments (one negative)
    n, incx, incy = 9, -2, 3
    xs = x[:o.blas_span(n, incx):2][::-1]
    want = y.copy()
    want[0:o.blas_span(n, incy):3] = alpha * xs + y[0:o.blas_span(n, incy):3]
    assert np.array_equal(bits64(o.axpy_strided(n, alpha, x, incx, y, incy, "f64")), bits64(want))
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    want32 = y32.copy()
    want32[0:o.blas_span(n, incy):3] = np.float32(alpha) * x32[:o.blas_span(n, incx):2][::-1] + \
        y32[0:o.blas_span(n, incy):3]
    assert np.array_equal(bits32(o.axpy_strided(n, alpha, x32, incx, y32, incy, "f32")), bits32(want32))


def check_asum(o):
    """asum: integers sum exactly; random values against math.fsum of |x|
    (correctly rounded) within the Dot2 bound."""
    v = np.array([3.0, -4.0, 0.0, -1.0, 2.0])
    assert o.asum(v)[0] == 10.0
    rng = np.random.default_rng(47)
    for n in (1, 17, 1000):
        x = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
        exact = math.fsum(abs(float(t)) for t in x)
        got = o.asum(x)[0]
        assert abs(got - exact) <= dot2_bound(n, exact, exact), (n, got, exact)


def check_reduce_canonical(o):
    """The replay of the library's summation order (a reading: the paper
    leaves the order open). Pins: hand-worked inputs whose result depends on
    the order -- each value below is derived by hand from the order's
    definition (tiles of 256 lanes x 16 chunks x V elements, lane l taking
    chunks l, l+256, ...; slot p per element of a chunk; butterflies over 64
    lanes; (g0 + g1) + (g2 + g3); a pairwise tree over the final combine's
    16 groups) and differs from what a sequential sum gives --, exact
    integer sums (exact in any order), and the Dot2 bound on random data."""
    big = 2.0 ** 53
    T64 = 256 * 16 * 2

    def dot64(x):
        return float(o.reduce_canonical("dot", x, np.ones(len(x)), "f64"))

    # slot separation and the lane's chunk stride: elements 0 and 512 are
    # lane 0's chunks 0 and 256 (slot 0), element 1 is slot 1: the slot-0 sum
    # 2^60 - 2^60 is exact and the slot-1 value 1 survives (sequentially the
    # 1 would be lost in 2^60 + 1)
    x = np.zeros(T64)
    x[0], x[1], x[512] = 2.0 ** 60, 1.0, -(2.0 ** 60)
    assert dot64(x) == 1.0
    assert o.naive_dot(x, np.ones(T64)) == 0.0
    # butterfly inside a group of 64 lanes: lanes 0, 2, 3 hold 2^53, 1, 1
    # (elements 0, 4, 6): (v0 + v1) + (v2 + v3) = 2^53 + 2; sequential 2^53
    x = np.zeros(T64)
    x[0], x[4], x[6] = big, 1.0, 1.0
    assert dot64(x) == big + 2
    # the four groups: lanes 0, 128, 192 -> (g0 + g1) + (g2 + g3) = 2^53 + 2
    x = np.zeros(T64)
    x[0], x[256], x[384] = big, 1.0, 1.0
    assert dot64(x) == big + 2
    # the final combine's butterfly: tiles 0, 2, 3 (its lanes 0, 2, 3)
    x = np.zeros(4 * T64)
    x[0], x[2 * T64], x[3 * T64] = big, 1.0, 1.0
    assert dot64(x) == big + 2
    # the final combine's pairwise tree over its 16 groups: tiles 0, 128,
    # 192 sit in groups 0, 2, 3 -> (g0 + g1) + (g2 + g3) = 2^53 + 2
    x = np.zeros(193 * T64)
    x[0], x[128 * T64], x[192 * T64] = big, 1.0, 1.0
    assert dot64(x) == big + 2
    # compensated binary32 slots keep the 1 that 2^30 + 1 rounds away (one
    # slot: elements 0, 1024, 2048 are lane 0's chunks 0, 256, 512, slot 0)
    for dt, hi, lo in (("f32", 2.0 ** 30, 1.0), ("bf16", 2.0 ** 30, 1.0), ("f16", 2.0 ** 15, 2.0 ** -9)):
        V = 4 if dt == "f32" else 8
        xs = np.zeros(256 * 16 * V, np.float32)
        xs[0], xs[256 * V], xs[512 * V] = hi, lo, -hi
        xs = xs if dt == "f32" else o.narrow(xs, dt)
        ones = np.ones(len(xs), np.float32)
        ones = ones if dt == "f32" else o.narrow(ones, dt)
        assert float(o.reduce_canonical("dot", xs, ones, dt)) == lo, dt
    # exact integer sums, every type, mode and a ragged tail
    for dt, V in (("f64", 2), ("f32", 4), ("bf16", 8), ("f16", 8)):
        T = 256 * 16 * V
        for n in (0, 1, 5, T - 1, T + 1, 3 * T + 5):
            i = np.arange(n, dtype=np.int64)
            xi, yi = i % 7 - 3, i % 5 - 2
            xs = xi.astype(np.float64) if dt == "f64" else xi.astype(np.float32)
            ys = yi.astype(np.float64) if dt == "f64" else yi.astype(np.float32)
            if dt in ("bf16", "f16"):
                xs, ys = o.narrow(xs, dt), o.narrow(ys, dt)
            rt = np.float64 if dt == "f64" else np.float32
            assert o.reduce_canonical("dot", xs, ys, dt) == rt(int((xi * yi).sum())), (dt, n)
            assert o.reduce_canonical("asum", xs, None, dt) == rt(int(np.abs(xi).sum())), (dt, n)
            assert o.reduce_canonical("nrm2", xs, None, dt) == rt(math.sqrt(int((xi * xi).sum()))), (dt, n)
        ones = np.ones(4 ** 8, np.float64 if dt == "f64" else np.float32)
        ones = ones if dt in ("f64", "f32") else o.narrow(ones, dt)
        assert float(o.reduce_canonical("nrm2", ones, None, dt)) == 256.0, dt
    # random values: within the tolerance of Dot2 on the stored values
    for dt, V in (("f64", 2), ("f32", 4), ("bf16", 8), ("f16", 8)):
        n = 3 * 256 * 16 * V + 17
        xs, ys = workloads.uniform(n, dt, 77, 2)
        xw, yw = o.widen(xs, dt), o.widen(ys, dt)
        ref, sabs = o.dot2(xw, yw)
        assert abs(float(o.reduce_canonical("dot", xs, ys, dt)) - ref) <= o.TOL[dt] * sabs, dt
        nref = o.nrm2(xw)
        assert abs(float(o.reduce_canonical("nrm2", xs, None, dt)) - nref) <= o.TOL[dt] * nref, dt
        aref = math.fsum(np.abs(xw).tolist())
        assert abs(float(o.reduce_canonical("asum", xs, None, dt)) - aref) <= o.TOL[dt] * aref, dt


def check_iamax(o):
    """iamax against numpy argmax of |x| (first occurrence of the maximum) and
    hand-worked cases: ties, NaNs, strides, empty vectors."""
    rng = np.random.default_rng(53)
    for dtype in ("f64", "f32"):
        for n in (1, 2, 33, 500):
            x = rng.standard_normal(3 * n)
            if dtype == "f32":
                x = x.astype(np.float32)
            for inc in (1, 3):
                want = int(np.argmax(np.abs(x[:o.blas_span(n, inc):inc])))
                assert o.iamax(n, x, inc, dtype) == want, (dtype, n, inc)
    t = np.array([1.0, -3.0, 3.0, 2.0, -3.0])
    assert o.iamax(5, t, 1, "f64") == 1                       # ties: the first
    assert o.iamax(3, t, 2, "f64") == 1                       # elements 1, 3, 3
    nan = float("nan")
    assert o.iamax(4, np.array([1.0, nan, 5.0, -5.0]), 1, "f64") == 2   # a NaN is skipped
    assert o.iamax(3, np.array([nan, 9.0, 1.0]), 1, "f64") == 0          # NaN first: kept
    assert o.iamax(3, np.array([0.0, -0.0, 0.0]), 1, "f64") == 0
    assert o.iamax(0, t, 1, "f64") == -1 and o.iamax(3, t, 0, "f64") == -1
    assert o.iamax(3, t, -1, "f64") == -1
    # 16-bit storage compares exact values: bfloat16 3.0 vs its neighbour 3.015625
    hb = o.narrow(np.array([3.0, -3.015625, 3.0], np.float32), "bf16")
    assert o.iamax(3, hb, 1, "bf16") == 1
    hf = o.narrow(np.array([1.0, 65504.0, -65504.0], np.float32), "f16")
    assert o.iamax(3, hf, 1, "f16") == 1


def check_h16_double_rounding(o):
    """The last operation of a 16-bit tree is rounded to binary32, then the
    result narrowed once (two roundings), not rounded from the exact value
    straight to 16 bits: a scalar multiple chosen so that the two differ on
    many inputs, against numpy (binary16) and torch (bfloat16) conversions
    of the binary32 products."""
    import torch

    alpha = 1.9255319833755493
    a32 = np.float32(alpha)
    x = np.arange(0x0400, 0x7800, dtype=np.uint16)             # positive binary16 normals below 2^15
    xf = x.view(np.float16).astype(np.float32)
    prog = [tok(SCALAR, 0), tok(LOAD, 0), tok(MUL)]
    exact = xf.astype(np.float64) * float(a32)
    twice = (xf * a32).astype(np.float16)
    assert np.count_nonzero(exact.astype(np.float16) != twice) >= 50    # one rounding differs here
    got = o.eval_program(prog, [x], [alpha], "f16")
    assert np.array_equal(np.asarray(got).view(np.uint16), twice.view(np.uint16))
    # bfloat16: all bfloat16 values in [0.5, 2), the binary32 product rounded by torch
    xb = np.arange(0x3f00, 0x4000, dtype=np.uint16)
    xbf = torch.from_numpy(xb.view(np.int16)).view(torch.bfloat16).to(torch.float32)
    want = (xbf * torch.tensor(a32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = o.eval_program(prog, [xb], [alpha], "bf16")
    assert np.array_equal(np.asarray(got).view(np.uint16), want)


CHECKS = {
    "h16_double_rounding": check_h16_double_rounding,
    "fig1_golden": check_fig1_golden,
    "python_float_trees_f64": check_python_float_trees_f64,
    "random_programs_f64": lambda o: check_random_programs(o, "f64"),
    "random_programs_f32": lambda o: check_random_programs(o, "f32"),
    "closed_form": check_closed_form,
    "invariants_f64": lambda o: check_invariants(o, "f64"),
    "invariants_f32": lambda o: check_invariants(o, "f32"),
    "f32_numpy_trees": check_f32_numpy_trees,
    "subnormals": check_subnormals,
    "rounding_golden": check_rounding_golden,
    "conversions_vs_libraries": check_conversions_vs_libraries,
    "h16_eval_bf16": lambda o: check_h16_eval_composition(o, "bf16"),
    "h16_eval_f16": lambda o: check_h16_eval_composition(o, "f16"),
    "axpy": check_axpy,
    "dot_closed_form": check_dot_closed_form,
    "dot_fraction_bruteforce": check_dot_fraction_bruteforce,
    "dot_fsum": check_dot_fsum,
    "nrm2": check_nrm2,
    "naive_f32": check_naive_f32,
    "naive_f64": check_naive_f64,
    "naive_par": check_naive_par,
    "eval_threads": check_eval_threads,
    "blas_strides": check_blas_strides,
    "scal_axpy_strided": check_scal_axpy_strided,
    "asum": check_asum,
    "iamax": check_iamax,
    "reduce_canonical": check_reduce_canonical,
}


@pytest.mark.parametrize("name", sorted(CHECKS))
def test_oracle_pin(orc, name):
    CHECKS[name](orc)


def test_oracle_rejects_bad_programs(orc):
    a = np.zeros(4)
    for prog in ([tok(ADD)], [tok(LOAD, 0), tok(LOAD, 0)], [tok(LOAD, 3)], [tok(SCALAR, 0)], [9]):
        with pytest.raises(ValueError):
            orc.eval_program(prog, [a], [], "f64")
