"""The expression front end (paper_1109_1264_amd.expr) on the host: operator
trees become the library's postfix programs, with the catalogue's exact
token streams for the catalogue trees, shared operands and scalars counted
once, the limits enforced before anything runs, and the stack-saving
exchange of addition and multiplication operands leaving every bit of the
result as the tree wrote it (checked with the oracle on the CPU). Programs
are built from CPU tensors: nothing is launched here."""
from __future__ import annotations

import random

import numpy as np
import pytest
import torch

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from paper_1109_1264_amd.expr import (Node, Scalar, Vec, dot, expression, norm, operand_key, pair_program,
                                      program, stack_need)

T = S.token


def vecs(k, n=16, dtype=torch.float64):
    return [Vec(torch.zeros(n, dtype=dtype)) for _ in range(k)]


def test_catalogue_trees_written_as_expressions():
    a, b, c, e, f, g = vecs(6)
    cat = dict(S.salt_catalogue())
    alpha = 1.5
    written = {
        "copy": a,
        "scale": alpha * a,
        "fig1": a + (b - c),
        "axpy": alpha * a + b,
        "tree5": a * b + c * e - f,
        "abc": alpha * a + (b - c),
        "t4": alpha * (a + b) - c * e,
        "t5": ((a * b + c) * (e - f)) + alpha * g,
    }
    assert set(written) == set(cat)
    for name, ex in written.items():
        p = program(ex)
        assert p.tokens == cat[name], name
        assert S.salt_program_route(p.tokens, len(p.operands), len(p.scalars)) >= 0, name


def test_operands_and_scalars_are_numbered_by_first_use_and_shared():
    a, b = vecs(2)
    p = program(2.0 * a + 2.0 * b - a)
    assert p.tokens == [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL), T(S.SCALAR, 0), T(S.LOAD, 1), T(S.MUL),
                        T(S.ADD), T(S.LOAD, 0), T(S.SUB)]
    assert p.scalars == [2.0] and len(p.operands) == 2
    # two wrappers of one tensor are one operand; a view of another range is not
    t = torch.zeros(32, dtype=torch.float64)
    p = program(Vec(t[:16]) + Vec(t[:16]) * Vec(t[16:]))
    assert len(p.operands) == 2 and p.tokens[:2] == [T(S.LOAD, 0), T(S.LOAD, 0)]
    # scalars by their bits: -0.0 and 0.0 are two scalars
    p = program(0.0 * a + (-0.0) * a)
    assert p.scalars == [0.0, -0.0] and np.signbit(p.scalars[1])
    # negation is a multiplication by -1; numbers on either side
    assert program(-a).tokens == [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL)] and program(-a).scalars == [-1.0]
    p = program(1 - a * 3)
    assert p.tokens == [T(S.SCALAR, 0), T(S.LOAD, 0), T(S.SCALAR, 1), T(S.MUL), T(S.SUB)]
    assert p.scalars == [1.0, 3.0]
    # raw tensors on the right of an expression are wrapped
    assert program(a + torch.zeros(16, dtype=torch.float64)).tokens == [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD)]


def test_limits_and_errors_before_any_launch():
    a, b = vecs(2)
    with pytest.raises(TypeError):
        program(a + Vec(torch.zeros(16, dtype=torch.float32)))      # two element types
    with pytest.raises(ValueError):
        program(a + Vec(torch.zeros(17, dtype=torch.float64)))      # two lengths
    many = vecs(9)
    ex = many[0]
    for v in many[1:]:
        ex = ex + v
    with pytest.raises(ValueError, match="at most 8 distinct vectors"):
        program(ex)
    ex = a
    for k in range(9):
        ex = ex + float(k + 1)
    with pytest.raises(ValueError, match="at most 8 distinct scalars"):
        program(ex)
    ex = a
    for _ in range(40):
        ex = ex + b
    with pytest.raises(ValueError, match="more than 64 tokens"):
        program(ex)
    s = a * b
    for _ in range(40):                                             # a DAG that expands past any limit
        s = s * s
    with pytest.raises(ValueError, match="more than 64 tokens"):
        program(s)
    with pytest.raises(ValueError):
        Vec(torch.zeros(4, 4, dtype=torch.float64))                 # not 1-D
    with pytest.raises(ValueError):
        Vec(torch.zeros(8, dtype=torch.float64)[::2])              # not unit stride
    with pytest.raises(TypeError):
        Vec(torch.zeros(8, dtype=torch.int32))                      # no such element type
    with pytest.raises(TypeError, match="unsupported tensor dtype"):
        a + torch.zeros(16, dtype=torch.int32)                      # the tensor's own error, not a generic one
    with pytest.raises(ValueError, match="1-D"):
        a + torch.zeros(4, 4, dtype=torch.float64)
    with pytest.raises(TypeError):
        a / b                                                       # not an operation of the method
    with pytest.raises(TypeError):
        a + "x"
    with pytest.raises(TypeError):
        bool(a + b)
    with pytest.raises(IndexError):
        a[1:] = b
    with pytest.raises(ValueError):
        Scalar(2.0).eval()                                          # no length
    with pytest.raises(ValueError):
        dot(Scalar(1.0), Scalar(2.0))
    with pytest.raises(ValueError):
        norm(Scalar(1.0) + 2.0)
    # the output is checked against the vectors before anything runs
    with pytest.raises(TypeError):
        program(a + b).check_output(torch.zeros(16, dtype=torch.float32))
    with pytest.raises(ValueError):
        program(a + b).check_output(torch.zeros(15, dtype=torch.float64))


def right_deep(leaves, ops):
    ex = leaves[-1]
    for v, op in zip(reversed(leaves[:-1]), reversed(ops)):
        ex = Node(op, v, ex)
    return ex


def natural_tokens(ex, p):
    """Left-first postfix of `ex` with p's operand and scalar numbering."""
    out = []

    def walk(e):
        if isinstance(e, Vec):
            out.append(T(S.LOAD, p._ops[operand_key(e.tensor)]))
        elif isinstance(e, Scalar):
            out.append(T(S.SCALAR, p.scalars.index(e.value)))
        else:
            walk(e.left)
            walk(e.right)
            out.append(T(e.op))
    walk(ex)
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_deep_trees_are_reordered_to_fit_with_the_same_bits(dtype):
    """A right-deep tree needs one stack slot per level as written; with the
    operands of + and * exchanged it needs two. The oracle (stack of 64)
    evaluates both programs: every element has the same bits."""
    rng = random.Random(11)
    n = 4099
    host = workloads.uniform(n, dtype, 1109, 6)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    leaves = [Vec(torch.zeros(n, dtype=tdt)) for _ in range(6)]
    checked = 0
    for trial in range(6):
        k = 12
        picks = [leaves[rng.randrange(6)] if rng.random() < 0.8 else Scalar(rng.choice([0.5, -1.25, 3.0]))
                 for _ in range(k)]
        if not any(isinstance(x, Vec) for x in picks):
            picks[0] = leaves[0]
        ops = [rng.choice([S.ADD, S.MUL, S.ADD, S.SUB]) for _ in range(k - 1)]
        ops[-1] = S.ADD                                   # the innermost level can always be exchanged
        ex = right_deep(picks, ops)
        p = program(ex)
        nat = natural_tokens(ex, p)
        assert stack_need(nat) > S.MAX_STACK or p.tokens == nat
        assert stack_need(p.tokens) <= S.MAX_STACK or S.SUB in ops
        assert sorted(p.tokens) == sorted(nat)            # the same tokens, some subtrees exchanged
        if stack_need(p.tokens) > S.MAX_STACK:
            continue                                      # subtractions pin the order: the library rejects it
        S.salt_program_check(p.tokens, len(p.operands), len(p.scalars))
        ops_host = [host[next(k for k, v in enumerate(leaves) if v.tensor is t)] for t in p.operands]
        got = oracle.eval_program(p.tokens, ops_host, p.scalars, dtype)
        want = oracle.eval_program(nat, ops_host, p.scalars, dtype)
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (trial, ex)
        checked += 1
    assert checked >= 3


def test_dot_pairs_leave_a_slot_for_the_other_value():
    """dot(P, Q) needs one of the two programs in 7 slots: a pair of two
    trees that need 8 as written has its first tree reordered, and the
    library's pair validation accepts it."""
    v = vecs(8)
    deep = v[0] + (v[1] + (v[2] + (v[3] + (v[4] + (v[5] + (v[6] + v[7]))))))
    also_deep = v[7] * (v[6] * (v[5] * (v[4] * (v[3] * (v[2] * (v[1] * v[0]))))))
    p0 = program(deep, also_deep)
    assert stack_need(p0.tokens) == 8 and stack_need(p0.tokens2) == 8
    p = pair_program(deep, also_deep)
    assert stack_need(p.tokens) == 2 and p.tokens2 == natural_tokens(also_deep, p)
    S.salt_reduce_expr_route(p.tokens, p.tokens2, len(p.operands), len(p.scalars))   # raises if rejected
    with pytest.raises(S.SaltError):
        S.salt_reduce_expr_route(p0.tokens, p0.tokens2, len(p0.operands), len(p0.scalars))
    # subtractions cannot be exchanged: the pair stays as written and is rejected
    sub = v[0] - (v[1] - (v[2] - (v[3] - (v[4] - (v[5] - (v[6] - v[7]))))))
    p = pair_program(sub, sub)
    assert stack_need(p.tokens) == 8
    with pytest.raises(S.SaltError):
        S.salt_reduce_expr_route(p.tokens, p.tokens2, len(p.operands), len(p.scalars))
    # a shallow pair keeps its order
    p = pair_program(v[0] + v[1], v[0] - v[1])
    assert p.tokens == [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD)]
    assert p.tokens2 == [T(S.LOAD, 0), T(S.LOAD, 1), T(S.SUB)]


def test_expressions_built_once():
    """expression(fn): the tree of a function of placeholder parameters,
    built once. Vector parameters load by position, scalar parameters come
    first among the scalars and the literals after them; the catalogue trees
    give the catalogue's token streams."""
    cat = dict(S.salt_catalogue())
    assert expression(lambda a, b, c: a + (b - c)).tokens == cat["fig1"]
    assert expression(lambda a, b, c, e, f: a * b + c * e - f).tokens == cat["tree5"]
    ax = expression(lambda x, y, alpha: alpha * x + y, scalars=("alpha",))
    assert ax.tokens == cat["axpy"] and ax.literals == [] and ax.is_scalar == [False, False, True]
    # literals are numbered after the scalar parameters; parameter order is
    # the load order whatever the order of use
    g = expression(lambda b, a, s: (a - b) * s + 0.5 * a - 0.5, scalars=("s",))
    assert g.tokens == [T(S.LOAD, 1), T(S.LOAD, 0), T(S.SUB), T(S.SCALAR, 0), T(S.MUL), T(S.SCALAR, 1),
                        T(S.LOAD, 1), T(S.MUL), T(S.ADD), T(S.SCALAR, 1), T(S.SUB)]
    assert g.literals == [0.5]
    S.salt_program_check(g.tokens, 2, 1 + len(g.literals))
    pair = expression(lambda a, b: (a + b, a - b))
    assert pair.pair and pair.tokens == [T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD)]
    assert pair.tokens2 == [T(S.LOAD, 0), T(S.LOAD, 1), T(S.SUB)]
    assert S.salt_reduce_expr_route(pair.tokens, pair.tokens2, 2, 0) == 0     # the catalogue pair
    # a deep tree is reordered as in the operator form
    deep = expression(lambda a, b: a + (b + (a + (b + (a + (b + (a + (b + (a + b)))))))))
    assert stack_need(deep.tokens) <= S.MAX_STACK
    # errors, all before anything runs
    with pytest.raises(ValueError):
        expression(lambda a: a * 2, scalars=("alpha",))                  # no such parameter
    with pytest.raises(ValueError):
        expression(lambda a, b, c: (a, b, c))                             # three trees
    x = Vec(torch.zeros(8, dtype=torch.float64))
    with pytest.raises(TypeError):
        expression(lambda a: a + x)                                       # a captured vector
    with pytest.raises(ValueError):
        expression(lambda a0, a1, a2, a3, a4, a5, a6, a7, a8: a0)         # nine vector parameters
    fig1 = expression(lambda a, b, c: a + (b - c))
    t = [torch.zeros(8, dtype=torch.float64) for _ in range(3)]
    with pytest.raises(TypeError):
        fig1(t[0], t[0], t[1])                                            # too few arguments
    with pytest.raises(ValueError):
        fig1(t[0], t[0], t[1], torch.zeros(9, dtype=torch.float64))      # two lengths
    with pytest.raises(ValueError):
        fig1(torch.zeros(9, dtype=torch.float64), *t)                    # output length
    with pytest.raises(TypeError):
        fig1.dot(*t)                                                      # not a pair
    with pytest.raises(TypeError):
        pair(t[0], t[1], t[2])                                            # a pair has no single value
    with pytest.raises(TypeError):
        pair.norm(t[0], t[1])


def test_expression_batches_check_their_items_first():
    """expression(...).batch: a pair cannot be batched; an empty list, a
    dots list of the wrong length, two element types or a wrong output
    length are refused before any plan is made."""
    f = expression(lambda a, b: a - b)
    pair = expression(lambda a, b: (a + b, a - b))
    t64 = [torch.zeros(8, dtype=torch.float64) for _ in range(3)]
    t32 = [torch.zeros(8, dtype=torch.float32) for _ in range(3)]
    with pytest.raises(TypeError):
        pair.batch([(t64[0], t64[1], t64[2])])
    with pytest.raises(ValueError):
        f.batch([])
    with pytest.raises(ValueError):
        f.batch([(t64[0], t64[1], t64[2])], dots=[None, None])
    with pytest.raises(TypeError):
        f.batch([(t64[0], t64[1], t64[2]), (t32[0], t32[1], t32[2])])
    with pytest.raises(ValueError):
        f.batch([(torch.zeros(9, dtype=torch.float64), t64[1], t64[2])])
