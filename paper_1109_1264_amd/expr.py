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

Building the tree costs host time on every statement (tens of
microseconds in Python). ``expression(fn)`` builds it once from a function
of placeholder parameters, the counterpart of C++'s compile-time expression
types; each call then costs one library call's marshalling.

Example::

    from paper_1109_1264_amd.expr import Vec, dot, expression, norm
    a, b, c, d = (Vec(t) for t in (ta, tb, tc, td))   # 1-D GPU tensors, one dtype
    d[:] = a + (b - c)            # Fig. 1: one kernel, one pass over memory
    d[:] = 2.5 * a + d            # axpy, in place
    r = dot(a + b, a - b)         # device scalar; a + b and a - b are never stored
    fig1 = expression(lambda a, b, c: a + (b - c))
    fig1(td, ta, tb, tc)          # the same call, tree built once
"""
from __future__ import annotations

import numbers
import struct
from typing import Sequence

from . import salt as S

__all__ = ["Expr", "Vec", "Scalar", "Param", "Node", "expression", "Program", "program", "pair_program",
           "operand_key", "stack_need", "dot", "norm"]

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


class Param(Expr):
    """A leaf of a tree built once by `expression`: the vector or scalar
    passed in that position of each call."""

    __slots__ = ("slot", "scalar", "name")

    def __init__(self, slot, scalar, name):
        self.slot, self.scalar, self.name = slot, scalar, name

    def __repr__(self):
        return self.name


class Node(Expr):
    """An operation: op in (ADD, SUB, MUL) applied to two subtrees."""

    __slots__ = ("op", "left", "right")

    def __init__(self, op, left, right):
        self.op, self.left, self.right = op, left, right

    def __repr__(self):
        return "(%r %s %r)" % (self.left, _SYMBOL[self.op], self.right)


def _leaf(x):
    """x as a tree node, or None for a type that takes no part in trees."""
    if isinstance(x, Expr):
        return x
    if isinstance(x, numbers.Real) and not isinstance(x, bool):
        return Scalar(x)
    if hasattr(x, "data_ptr") and hasattr(x, "dim"):
        return Vec(x)  # raises for a tensor the library cannot take
    return None


def _as_expr(x) -> Expr:
    e = _leaf(x)
    if e is None:
        raise TypeError("cannot use %s in a vector expression" % type(x).__name__)
    return e


def _node(op, left, right):
    l, r = _leaf(left), _leaf(right)
    if l is None or r is None:
        return NotImplemented  # Python then tries the other operand, or raises TypeError
    return Node(op, l, r)


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


def operand_key(t):
    """Vectors are one operand when they are the same memory: start, length,
    element type and device."""
    return (t.data_ptr(), t.numel(), t.dtype, t.get_device())


class Program:
    """Trees over one shared list of operands and scalars, as the library's
    postfix programs: `tokens` for the first tree (and `tokens2` for a
    second, as a dot product takes)."""

    def __init__(self):
        self.operands = []   # torch tensors, LOAD k reads operands[k]
        self.scalars = []    # floats, SCALAR j reads scalars[j]
        self._ops = {}
        self._keys = []      # operand_key of each operand
        self._seen = {}      # id(tensor) -> operand index (tensors are held in operands)
        self._scs = {}
        self.tokens = []
        self.tokens2 = None
        self.template = False  # built by expression(): leaves are Params and literals
        self.params = 0        # scalar parameters ahead of the literals (expression())

    def _operand(self, v: Vec) -> int:
        if self.template:
            raise TypeError("a tree built by expression() takes its vectors as parameters, not %r" % (v,))
        t = v.tensor
        k = self._seen.get(id(t))
        if k is not None:
            return k
        key = operand_key(t)
        k = self._ops.get(key)
        if k is None:
            if self.operands:
                ref = self._keys[0]
                if key[2] != ref[2]:
                    raise TypeError("vectors of one expression must share a dtype (%s and %s)" % (ref[2], key[2]))
                if key[1] != ref[1]:
                    raise ValueError("vectors of one expression must have one length (%d and %d)" % (ref[1], key[1]))
                if key[3] != ref[3]:
                    raise ValueError("vectors of one expression must be on one device")
            if len(self.operands) == S.MAX_OPERANDS:
                raise ValueError("an expression reads at most %d distinct vectors" % S.MAX_OPERANDS)
            k = self._ops[key] = len(self.operands)
            self.operands.append(t)
            self._keys.append(key)
        self._seen[id(t)] = k
        return k

    def _scalar(self, s: Scalar) -> int:
        key = struct.pack("<d", s.value)  # by bits: -0.0 and 0.0 stay apart
        if key not in self._scs:
            if self.params + len(self.scalars) == S.MAX_SCALARS:
                raise ValueError("an expression uses at most %d distinct scalars" % S.MAX_SCALARS)
            self._scs[key] = self.params + len(self.scalars)
            self.scalars.append(s.value)
        return self._scs[key]

    def _emit(self, root: Expr, memo) -> list:
        """Postfix of `root`: left operand first, or (memo a dict) with the
        side that needs more stack first in additions and multiplications.
        Stops as soon as the tree is too large: past MAX_TOKENS tokens, or
        nested deeper than a tree of MAX_TOKENS tokens can be."""
        out = []
        cap = S.MAX_TOKENS

        def too_large():
            return ValueError("an expression expands to more than %d tokens" % cap)

        def walk(e, depth):
            if isinstance(e, Vec):
                out.append(S.token(S.LOAD, self._operand(e)))
            elif isinstance(e, Scalar):
                out.append(S.token(S.SCALAR, self._scalar(e)))
            elif isinstance(e, Param):
                out.append(S.token(S.SCALAR if e.scalar else S.LOAD, e.slot))
            else:
                if 2 * depth + 3 > cap:  # this node, a leaf beside each ancestor
                    raise too_large()
                first, second = e.left, e.right
                if memo is not None and e.op != S.SUB and _need(second, True, memo) > _need(first, True, memo):
                    first, second = second, first
                walk(first, depth + 1)
                walk(second, depth + 1)
                out.append(S.token(e.op))
            if len(out) > cap:
                raise too_large()

        walk(root, 0)
        return out

    def add(self, root: Expr, limit: int = None) -> list:
        """Tokens of one tree (as written; reordered when that needs more
        than `limit` stack slots, MAX_STACK by default)."""
        root = _as_expr(root)
        tokens = self._emit(root, None)
        if stack_need(tokens) > (S.MAX_STACK if limit is None else limit):
            tokens = self._emit(root, {})
        return tokens

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


def pair_program(x, y, params: int | None = None) -> Program:
    """The programs of dot(x, y) over one operand list. One of the two must
    leave a stack slot for the other's value: the trees as written, else the
    first and then the second held to one slot less (by exchanging operands
    of additions and multiplications); the library rejects a pair that still
    does not fit."""
    x, y = _as_expr(x), _as_expr(y)
    for lx, ly in ((None, None), (S.MAX_STACK - 1, None), (None, S.MAX_STACK - 1)):
        p = Program()
        if params is not None:
            p.template, p.params = True, params
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


class expression:
    """A tree built once, from a function of its parameters, and evaluated
    by each call: the counterpart of the paper's compile-time expression
    types (Sec. 2). The tree, its postfix program and its scalar literals are
    fixed when the object is made; a call only hands the library its
    vectors, scalars and output, so its host cost is that of one salt_eval
    call whatever the tree's size.

    The function's parameters named in `scalars` are numbers, the others
    vectors (1-D GPU tensors or Vec, one element type and length per call).
    A function returning one tree evaluates into an output or takes its
    norm; one returning a pair (x, y) takes their dot product::

        fig1 = expression(lambda a, b, c: a + (b - c))
        fig1(d, ta, tb, tc)                      # d <- a + (b - c)
        axpy = expression(lambda x, y, alpha: alpha * x + y, scalars=("alpha",))
        axpy(ty, tx, ty, 2.5)                    # in place
        pair = expression(lambda a, b: (a + b, a - b))
        r = pair.dot(ta, tb)                     # device scalar
    """

    def __init__(self, fn, scalars: Sequence[str] = ()):
        import inspect

        names = list(inspect.signature(fn).parameters)
        unknown = set(scalars) - set(names)
        if unknown:
            raise ValueError("scalars names no parameter: %s" % sorted(unknown))
        self.names = names
        self.is_scalar = [n in scalars for n in names]
        nv = sum(1 for x in self.is_scalar if not x)
        ns = len(names) - nv
        if nv > S.MAX_OPERANDS or ns > S.MAX_SCALARS:
            raise ValueError("at most %d vector and %d scalar parameters" % (S.MAX_OPERANDS, S.MAX_SCALARS))
        slots, kv, ks = [], 0, 0
        for sc, n in zip(self.is_scalar, names):
            slots.append(Param(ks if sc else kv, sc, n))
            ks, kv = ks + sc, kv + (not sc)
        tree = fn(*slots)
        if isinstance(tree, tuple):
            if len(tree) != 2:
                raise ValueError("a dot product takes a pair of trees")
            p = pair_program(tree[0], tree[1], params=ns)
            self.pair = True
        else:
            p = Program()
            p.template, p.params = True, ns
            p.tokens = p.add(_as_expr(tree))
            self.pair = False
        self.tokens, self.tokens2, self.literals = p.tokens, p.tokens2, list(p.scalars)
        self.tree = tree

    def _split(self, args):
        if len(args) != len(self.names):
            raise TypeError("expected %d arguments (%s), got %d" % (len(self.names), ", ".join(self.names), len(args)))
        vecs, scs = [], []
        for sc, a in zip(self.is_scalar, args):
            if sc:
                scs.append(float(a))
            else:
                vecs.append(a.tensor if isinstance(a, Vec) else a)
        n = vecs[0].numel() if vecs else None
        for t in vecs:
            if t.numel() != n:
                raise ValueError("vectors of one call must have one length (%d and %d)" % (n, t.numel()))
        return vecs, scs + self.literals, n

    def __call__(self, out, *args, stream=None):
        """out <- the tree over these arguments, in one salt_eval call."""
        if self.pair:
            raise TypeError("a pair of trees has no single value: use .dot(...)")
        out = out.tensor if isinstance(out, Vec) else out
        vecs, scs, n = self._split(args)
        if n is not None and out.numel() != n:
            raise ValueError("output length %d differs from the vectors' %d" % (out.numel(), n))
        S.salt_eval(self.tokens, vecs, scs, out, n=out.numel(), stream=stream)
        return out

    def dot(self, *args, stream=None, result=None):
        """Device scalar sum_i x_i * y_i of the pair (one salt_dot_expr call)."""
        if not self.pair:
            raise TypeError("a dot product needs a function returning a pair (x, y)")
        vecs, scs, n = self._split(args)
        if n is None:
            raise ValueError("a dot product of scalars only has no length")
        return S.salt_dot_expr(self.tokens, self.tokens2, vecs, scs, n=n, result=result, stream=stream)

    def batch(self, items, dots=None, stream=None):
        """Many evaluations of this tree in one persistent launch: a batched
        plan (paper_1109_1264_amd.batch.Batch; launch it, or capture it in a
        graph) whose item k is items[k] = (out, *args), as for a call. The
        items may differ in length, vectors and scalars, not in element
        type. With `dots`, item k also computes into dots[k] (a one-element
        device tensor, or None) the dot product of its first two vector
        arguments, in the same pass, with the bits of salt_dot on them; the
        tree must read those two first, in that order (the plan refuses it
        otherwise)."""
        from .batch import Batch

        if self.pair:
            raise TypeError("a batch evaluates one tree per item")
        if not items:
            raise ValueError("a batch needs at least one item")
        if dots is not None and len(dots) != len(items):
            raise ValueError("one dot result (or None) per item")
        plan, dtype = [], None
        for k, item in enumerate(items):
            out = item[0].tensor if isinstance(item[0], Vec) else item[0]
            vecs, scs, n = self._split(item[1:])
            if n is not None and out.numel() != n:
                raise ValueError("item %d: output length %d differs from the vectors' %d" % (k, out.numel(), n))
            d = S.dtype_code(out)
            if dtype is None:
                dtype = d
            elif d != dtype:
                raise TypeError("the items of one batch share an element type")
            plan.append({"n": out.numel(), "operands": vecs, "scalars": scs, "out": out,
                         "dot_out": None if dots is None else dots[k]})
        return Batch(self.tokens, plan, dtype, stream=stream)

    def norm(self, *args, stream=None, result=None):
        """Device scalar sqrt(sum_i x_i^2) of the tree (one salt_nrm2_expr call)."""
        if self.pair:
            raise TypeError("the norm takes one tree")
        vecs, scs, n = self._split(args)
        if n is None:
            raise ValueError("the norm of scalars only has no length")
        return S.salt_nrm2_expr(self.tokens, vecs, scs, n=n, result=result, stream=stream)
