"""Expression objects over device vectors: the paper's expression templates
(Sec. 2) as the host-side front end of the library.

Operators on vectors and scalars (``+``, ``-``, ``*``, unary ``-``) return
tree nodes instead of computing anything. A tree is evaluated only where its
value is needed (lazy evaluation, Sec. 2):

- assigned to a vector: ``d[:] = a + (b - c)`` or ``d.assign(...)``;
- evaluated into a new tensor: ``(a * b + c * e - f).eval()``;
- reduced without being written: ``dot(a + b, a - b)``, ``norm(x - y)``.

Each of these is ONE call of the library. The whole tree becomes one postfix
program (each distinct vector one LOAD operand, each distinct scalar value
one SCALAR), which one fused kernel evaluates per element on the GPU
(salt_eval, salt_dot_expr, salt_nrm2_expr; plain vectors go to salt_dot and
salt_nrm2). Nothing here touches the data. The tree's shape is the order of
evaluation: the left operand of every operation comes first, and each
operation is rounded once in the element type's compute precision, as
salt_eval defines. A tree that needs more stack slots than a program may use
has the operands of its additions and multiplications exchanged where that
lowers the need (IEEE addition and multiplication are commutative, so every
result keeps its bits); a subtraction keeps its order.

Example::

    from paper_1109_1264_amd.expr import Vec, dot, norm
    a, b, c, d = (Vec(t) for t in (ta, tb, tc, td))   # 1-D GPU tensors, one dtype
    d[:] = a + (b - c)            # Fig. 1: one kernel, one pass over memory
    d[:] = 2.5 * a + d            # axpy, in place
    r = dot(a + b, a - b)         # device scalar; a + b and a - b are never stored
"""
from __future__ import annotations

import numbers
import struct
from typing import Sequence

from . import salt as S

__all__ = ["Expr", "Vec", "Scalar", "Node", "Program", "program", "pair_program", "stack_need", "dot", "norm"]

_SYMBOL = {S.ADD: "+", S.SUB: "-", S.MUL: "*"}


class Expr:
    """A node of an expression tree. Operators build larger trees; nothing
    is computed until the tree is assigned, evaluated or reduced."""

    __slots__ = ()

    def __add__(self, o):
        return _node(S.ADD, self, o)

    def __radd__(self, o):
        return _node(S.ADD, o, self)

    def __sub__(self, o):
        return _node(S.SUB, self, o)

    def __rsub__(self, o):
        return _node(S.SUB, o, self)

    def __mul__(self, o):
        return _node(S.MUL, self, o)

    def __rmul__(self, o):
        return _node(S.MUL, o, self)

    def __neg__(self):
        # multiplying by -1 flips the sign bit and nothing else
        return _node(S.MUL, Scalar(-1.0), self)

    def __bool__(self):
        raise TypeError("an expression has no truth value; assign, evaluate or reduce it first")

    def eval(self, out=None, stream=None):
        """Evaluate the tree into `out` (a 1-D GPU tensor; a new one when
        None) with one salt_eval call; returns the tensor."""
        p = program(self)
        if out is None:
            import torch

            if not p.operands:
                raise ValueError("a tree of scalars only has no length: pass `out`")
            ref = p.operands[0]
            out = torch.empty(ref.numel(), dtype=ref.dtype, device=ref.device)
        p.check_output(out)
        S.salt_eval(p.tokens, p.operands, p.scalars, out, n=out.numel(), stream=stream)
        return out


class Vec(Expr):
    """A leaf: a 1-D vector in device memory (a torch tensor with unit
    stride; float64, float32, bfloat16 or float16). Assigning an expression
    to it (``v[:] = expr``) evaluates the expression into its memory."""

    __slots__ = ("tensor",)

    def __init__(self, tensor):
        if tensor.dim() != 1 or (tensor.numel() > 1 and tensor.stride(0) != 1):
            raise ValueError("a vector must be a 1-D tensor with unit stride")
        S.dtype_code(tensor)  # raises for an element type the library does not have
        self.tensor = tensor

    def __len__(self):
        return self.tensor.numel()

    def __setitem__(self, key, value):
        if key != slice(None) and key is not Ellipsis:
            raise IndexError("only the whole vector can be assigned: v[:] = expression")
        self.assign(value)

    def assign(self, value, stream=None):
        """self <- value (an expression, a vector or a number), in one call."""
        _as_expr(value).eval(out=self.tensor, stream=stream)
        return self

    def __repr__(self):
        return "Vec(n=%d, %s)" % (self.tensor.numel(), self.tensor.dtype)


class Scalar(Expr):
    """A leaf: a real number, rounded once to the compute type when the
    tree is evaluated (binary64 for float64 vectors, binary32 otherwise)."""

    __slots__ = ("value",)

    def __init__(self, value):
        self.value = float(value)

    def __repr__(self):
        return repr(self.value)


class Node(Expr):
    """An operation: op in (ADD, SUB, MUL) applied to two subtrees."""

    __slots__ = ("op", "left", "right")

    def __init__(self, op, left, right):
        self.op, self.left, self.right = op, left, right

    def __repr__(self):
        return "(%r %s %r)" % (self.left, _SYMBOL[self.op], self.right)


def _as_expr(x) -> Expr:
    if isinstance(x, Expr):
        return x
    if isinstance(x, numbers.Real) and not isinstance(x, bool):
        return Scalar(x)
    if hasattr(x, "data_ptr") and hasattr(x, "dim"):
        return Vec(x)
    raise TypeError("cannot use %s in a vector expression" % type(x).__name__)


def _node(op, left, right):
    try:
        return Node(op, _as_expr(left), _as_expr(right))
    except TypeError:
        return NotImplemented


def _count_nodes(roots: Sequence[Expr], limit: int) -> int:
    """Tokens the trees expand to (a subtree used twice counts twice),
    stopping once past `limit`."""
    count, todo = 0, list(roots)
    while todo and count <= limit:
        e = todo.pop()
        count += 1
        if isinstance(e, Node):
            todo.append(e.left)
            todo.append(e.right)
    return count


def _need(e: Expr, swap: bool, memo: dict) -> int:
    """Stack slots the postfix of `e` needs (left operand first; with `swap`
    the larger side of an addition or multiplication goes first)."""
    k = id(e)
    if k in memo:
        return memo[k]
    if not isinstance(e, Node):
        v = 1
    else:
        nl, nr = _need(e.left, swap, memo), _need(e.right, swap, memo)
        if swap and e.op != S.SUB and nr > nl:
            nl, nr = nr, nl
        v = max(nl, nr + 1)
    memo[k] = v
    return v


class Program:
    """Trees over one shared list of operands and scalars, as the library's
    postfix programs: `tokens` for the first tree (and `tokens2` for a
    second, as a dot product takes)."""

    def __init__(self):
        self.operands = []   # torch tensors, LOAD k reads operands[k]
        self.scalars = []    # floats, SCALAR j reads scalars[j]
        self._ops = {}
        self._scs = {}
        self.tokens = []
        self.tokens2 = None

    def _operand(self, v: Vec) -> int:
        t = v.tensor
        key = (t.data_ptr(), t.numel(), t.dtype, str(t.device))
        if key not in self._ops:
            if self.operands:
                ref = self.operands[0]
                if t.dtype != ref.dtype:
                    raise TypeError("vectors of one expression must share a dtype (%s and %s)" % (ref.dtype, t.dtype))
                if t.numel() != ref.numel():
                    raise ValueError("vectors of one expression must have one length (%d and %d)"
                                     % (ref.numel(), t.numel()))
                if t.device != ref.device:
                    raise ValueError("vectors of one expression must be on one device")
            if len(self.operands) == S.MAX_OPERANDS:
                raise ValueError("an expression reads at most %d distinct vectors" % S.MAX_OPERANDS)
            self._ops[key] = len(self.operands)
            self.operands.append(t)
        return self._ops[key]

    def _scalar(self, s: Scalar) -> int:
        key = struct.pack("<d", s.value)  # by bits: -0.0 and 0.0 stay apart
        if key not in self._scs:
            if len(self.scalars) == S.MAX_SCALARS:
                raise ValueError("an expression uses at most %d distinct scalars" % S.MAX_SCALARS)
            self._scs[key] = len(self.scalars)
            self.scalars.append(s.value)
        return self._scs[key]

    def _emit(self, root: Expr, limit: int) -> list:
        swap = _need(root, False, {}) > limit
        memo = {} if swap else None
        out = []

        def walk(e):
            if isinstance(e, Vec):
                out.append(S.token(S.LOAD, self._operand(e)))
            elif isinstance(e, Scalar):
                out.append(S.token(S.SCALAR, self._scalar(e)))
            else:
                first, second = e.left, e.right
                if swap and e.op != S.SUB and _need(second, True, memo) > _need(first, True, memo):
                    first, second = second, first
                walk(first)
                walk(second)
                out.append(S.token(e.op))

        walk(root)
        return out

    def add(self, root: Expr, limit: int = None) -> list:
        root = _as_expr(root)
        if _count_nodes([root], S.MAX_TOKENS) > S.MAX_TOKENS:
            raise ValueError("an expression expands to more than %d tokens" % S.MAX_TOKENS)
        return self._emit(root, S.MAX_STACK if limit is None else limit)

    def check_output(self, out) -> None:
        if out.dim() != 1 or (out.numel() > 1 and out.stride(0) != 1):
            raise ValueError("the output must be a 1-D tensor with unit stride")
        if self.operands:
            ref = self.operands[0]
            if out.dtype != ref.dtype:
                raise TypeError("output dtype %s differs from the vectors' %s" % (out.dtype, ref.dtype))
            if out.numel() != ref.numel():
                raise ValueError("output length %d differs from the vectors' %d" % (out.numel(), ref.numel()))


def stack_need(tokens: Sequence[int]) -> int:
    """Largest number of values a postfix program holds on its stack."""
    depth = most = 0
    for t in tokens:
        depth += 1 if (t & 0xFF) in (S.LOAD, S.SCALAR) else -1
        most = max(most, depth)
    return most


def program(expr, expr2=None) -> Program:
    """The postfix program(s) of one tree, or of two trees over one operand
    list (a dot product's pair). Raises before anything runs when the trees
    mix element types or lengths, or exceed the library's limits."""
    p = Program()
    p.tokens = p.add(expr)
    if expr2 is not None:
        p.tokens2 = p.add(expr2)
    return p


def pair_program(x, y) -> Program:
    """The programs of dot(x, y) over one operand list. One of the two must
    leave a stack slot for the other's value: the trees as written, else the
    first and then the second held to one slot less (by exchanging operands
    of additions and multiplications); the library rejects a pair that still
    does not fit."""
    x, y = _as_expr(x), _as_expr(y)
    for lx, ly in ((None, None), (S.MAX_STACK - 1, None), (None, S.MAX_STACK - 1)):
        p = Program()
        p.tokens = p.add(x, lx)
        p.tokens2 = p.add(y, ly)
        if min(stack_need(p.tokens), stack_need(p.tokens2)) < S.MAX_STACK:
            break
    return p


def dot(x, y, stream=None, result=None):
    """Device scalar sum_i x_i * y_i of two expressions, in one pass: neither
    tree is stored (salt_dot_expr; salt_dot for two plain vectors).
    Binary64 for float64 vectors, binary32 otherwise."""
    x, y = _as_expr(x), _as_expr(y)
    p = pair_program(x, y)  # also checks element types and lengths
    if isinstance(x, Vec) and isinstance(y, Vec):
        return S.salt_dot(x.tensor, y.tensor, result=result, stream=stream)
    if not p.operands:
        raise ValueError("a dot product of scalars only has no length")
    return S.salt_dot_expr(p.tokens, p.tokens2, p.operands, p.scalars, result=result, stream=stream)


def norm(x, stream=None, result=None):
    """Device scalar sqrt(sum_i x_i^2) of an expression, in one pass
    (salt_nrm2_expr; salt_nrm2 for a plain vector)."""
    x = _as_expr(x)
    if isinstance(x, Vec):
        return S.salt_nrm2(x.tensor, result=result, stream=stream)
    p = program(x)
    if not p.operands:
        raise ValueError("the norm of scalars only has no length")
    return S.salt_nrm2_expr(p.tokens, p.operands, p.scalars, result=result, stream=stream)
