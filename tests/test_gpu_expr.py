"""The expression front end on the GPU: assignments, evaluations and
reductions written with operators go through one library call each and
match the oracle -- element-wise results bit for bit (the oracle evaluates
the tree as written, left operand first), dot and norm within the Dot2
tolerance and with the bits of the library's own calls on the same
programs. Lengths span several tiles with a ragged tail; one case per
element type uses unaligned views."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads
from paper_1109_1264_amd.expr import Node, Scalar, Vec, dot, expression, norm, operand_key, program, stack_need
from tests.gpu_util import BITS, CODE, first_mismatch, to_dev, to_host_bits

pytestmark = pytest.mark.gpu
T = S.token
DTYPES = ["f64", "f32", "bf16", "f16"]
N = 300007


def leaves(dtype, n, seed, count, offset=0):
    host = workloads.uniform(n, dtype, seed, count)
    return host, [Vec(to_dev(h, dtype, offset=offset)) for h in host]


def natural(ex, p):
    """Left-first postfix of `ex` in p's numbering (the tree as written)."""
    out = []

    def walk(e):
        if isinstance(e, Vec):
            out.append(T(S.LOAD, next(k for k, t in enumerate(p.operands) if operand_key(t) == operand_key(e.tensor))))
        elif isinstance(e, Scalar):
            out.append(T(S.SCALAR, p.scalars.index(e.value)))
        else:
            walk(e.left)
            walk(e.right)
            out.append(T(e.op))
    walk(ex)
    return out


def oracle_of(ex, host_of, dtype, n):
    p = program(ex)
    ops = [host_of[id(t)] for t in p.operands]
    return oracle.eval_program(natural(ex, p), ops, p.scalars, dtype, n=n)


def check_bits(out, want, dtype, what):
    got = to_host_bits(out, dtype)
    want = np.ascontiguousarray(want).view(BITS[dtype])
    assert np.array_equal(got, want), (what, first_mismatch(got, want))


@pytest.mark.parametrize("dtype", DTYPES)
def test_assignments_and_evaluations(dtype):
    import torch

    for offset in (0, 1):
        host, (a, b, c, e, f) = leaves(dtype, N, 1109 + offset, 5, offset)
        host_of = {id(v.tensor): h for v, h in zip((a, b, c, e, f), host)}
        d = Vec(to_dev(np.zeros_like(host[0]), dtype, offset=offset))
        alpha = workloads.alpha(1264)
        cases = [
            ("fig1", a + (b - c)),
            ("tree5", a * b + c * e - f),
            ("t5", ((a * b + c) * (e - f)) + alpha * a),
            ("outside the catalogue", (a - b) * (a + 0.5) - c * c + 3 * (e - -f)),
            ("scalars only", Scalar(0.1) * 3 - 1),
        ]
        for name, ex in cases:
            print("case", dtype, offset, name, flush=True)
            d[:] = ex
            torch.cuda.synchronize()
            if name == "scalars only":
                want = oracle.eval_program([T(S.SCALAR, 0), T(S.SCALAR, 1), T(S.MUL), T(S.SCALAR, 2), T(S.SUB)],
                                           [], [0.1, 3.0, 1.0], dtype, n=N)
            else:
                want = oracle_of(ex, host_of, dtype, N)
            check_bits(d.tensor, want, dtype, name)
        # .eval() allocates the output
        out = (a * b + c * e - f).eval()
        torch.cuda.synchronize()
        check_bits(out, oracle_of(a * b + c * e - f, host_of, dtype, N), dtype, "eval")
        # axpy in place: y <- alpha*x + y, one call, y read and written
        y_host = host[1].copy()
        y = Vec(to_dev(y_host, dtype, offset=offset))
        y[:] = alpha * a + y
        torch.cuda.synchronize()
        check_bits(y.tensor, oracle.axpy(alpha, host[0], y_host, dtype), dtype, "axpy in place")


@pytest.mark.parametrize("dtype", DTYPES)
def test_deep_trees_reordered_keep_the_bits(dtype):
    """A tree deeper than the library's 8 stack slots runs with operands of
    its additions and multiplications exchanged; every element has the bits
    of the oracle evaluating the tree as written."""
    import torch

    host, vs = leaves(dtype, N, 4242, 6)
    host_of = {id(v.tensor): h for v, h in zip(vs, host)}
    ex = vs[0]
    for k in range(11):                 # right-deep: needs 12 slots as written
        ex = Node(S.ADD if k % 3 else S.MUL, vs[(k + 1) % 6] if k % 4 else Scalar(0.5 + k), ex)
    ex = Node(S.SUB, ex, vs[5])
    p = program(ex)
    assert stack_need(natural(ex, p)) > S.MAX_STACK >= stack_need(p.tokens)
    out = ex.eval()
    torch.cuda.synchronize()
    check_bits(out, oracle_of(ex, host_of, dtype, N), dtype, "deep")


@pytest.mark.parametrize("dtype", DTYPES)
def test_dot_and_norm_of_expressions(dtype):
    import torch

    Tt = S.salt_reduce_tile_elems(CODE[dtype])
    for n in (0, 1, Tt - 3, 3 * Tt + 11, N):
        host, (a, b, c) = leaves(dtype, n, 77 + n % 101, 3)
        host_of = {id(v.tensor): h for v, h in zip((a, b, c), host)}
        pairs = [
            ("dot(a + b, a - b)", dot(a + b, a - b),
             S.salt_dot_expr([T(S.LOAD, 0), T(S.LOAD, 1), T(S.ADD)], [T(S.LOAD, 0), T(S.LOAD, 1), T(S.SUB)],
                             [a.tensor, b.tensor], [], n=n), (a + b, a - b)),
            ("dot(a, b)", dot(a, b), S.salt_dot(a.tensor, b.tensor, n=n), (a, b)),
            ("dot(2a*c, b)", dot(2.0 * a * c, b),
             S.salt_dot_expr([T(S.SCALAR, 0), T(S.LOAD, 0), T(S.MUL), T(S.LOAD, 1), T(S.MUL)], [T(S.LOAD, 2)],
                             [a.tensor, c.tensor, b.tensor], [2.0], n=n), (2.0 * a * c, b)),
            ("norm(a - b)", norm(a - b),
             S.salt_nrm2_expr([T(S.LOAD, 0), T(S.LOAD, 1), T(S.SUB)], [a.tensor, b.tensor], [], n=n), (a - b, None)),
            ("norm(c)", norm(c), S.salt_nrm2(c.tensor, n=n), (c, None)),
        ]
        torch.cuda.synchronize()
        for name, got, lib_call, (x, y) in pairs:
            print("case", dtype, n, name, flush=True)
            assert got.item() == lib_call.item(), (name, dtype, n, got.item(), lib_call.item())
            vx = oracle.widen(oracle_of(x, host_of, dtype, n), dtype)
            if y is None:
                ref, _ = oracle.dot2(vx, vx)
                assert abs(got.item() - np.sqrt(ref)) <= oracle.TOL[dtype] * np.sqrt(ref) + 1e-300, (name, n)
            else:
                vy = oracle.widen(oracle_of(y, host_of, dtype, n), dtype)
                ref, abs_sum = oracle.dot2(vx, vy)
                assert abs(got.item() - ref) <= oracle.TOL[dtype] * abs_sum + 1e-300, (name, n)


@pytest.mark.parametrize("dtype", DTYPES)
def test_expressions_built_once(dtype):
    """A tree built once by expression() and called with several argument
    sets has, every time, the bits of the same tree written with operators
    (checked against the oracle); its dot and norm have the bits of the
    operator forms."""
    import torch

    host, vs = leaves(dtype, N, 555, 3, offset=1)
    host_of = {id(v.tensor): h for v, h in zip(vs, host)}
    a, b, c = vs
    f = expression(lambda x, y, z, s: (x - y) * s + z * 0.75, scalars=("s",))
    out = Vec(to_dev(np.zeros_like(host[0]), dtype))
    for (x, y, z), s in (((a, b, c), 1.375), ((c, a, b), -2.5), ((b, b, a), 0.0)):
        print("case", dtype, s, flush=True)
        f(out, x.tensor, y, z.tensor, s)              # tensors or Vec
        torch.cuda.synchronize()
        check_bits(out.tensor, oracle_of((x - y) * s + z * 0.75, host_of, dtype, N), dtype, ("template", s))
    pair = expression(lambda x, y: (x + y, x - y))
    got = pair.dot(a, b)
    want = dot(a + b, a - b)
    nrm = f.norm(a, b, c, 1.375)
    want_nrm = norm((a - b) * 1.375 + c * 0.75)
    torch.cuda.synchronize()
    assert got.item() == want.item(), (got.item(), want.item())
    assert nrm.item() == want_nrm.item(), (nrm.item(), want_nrm.item())
    vx = oracle.widen(oracle_of(a + b, host_of, dtype, N), dtype)
    vy = oracle.widen(oracle_of(a - b, host_of, dtype, N), dtype)
    ref, abs_sum = oracle.dot2(vx, vy)
    assert abs(got.item() - ref) <= oracle.TOL[dtype] * abs_sum


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_expression_batch(dtype):
    """A built-once tree over 27 ragged items (aligned and not, each with its
    own scalar) as one batched launch and as a replayed graph: every output
    has the bits of the oracle evaluating the tree as written, and the fused
    dots those of salt_dot on the first two vector arguments (which the
    tree reads first). Empty items are part of the list."""
    import torch

    rng = np.random.default_rng(77)
    f = expression(lambda x, y, z, s: (x - y) * s + z * 0.75, scalars=("s",))
    lengths = [1, 0, 5, 100, 4099, 16387, 70001] + [int(v) for v in rng.integers(1, 40000, 20)]
    rdt = torch.float64 if dtype == "f64" else torch.float32
    items, dots, cases = [], [], []
    for k, n in enumerate(lengths):
        host = workloads.uniform(n, dtype, 6000 + k, 3)
        vs = [Vec(to_dev(h, dtype, offset=k % 2)) for h in host]
        out = to_dev(np.zeros_like(host[0]), dtype, offset=(k // 2) % 2)
        s = float(rng.uniform(-2, 2))
        items.append((out, vs[0], vs[1].tensor, vs[2], s))
        dots.append(torch.empty(1, dtype=rdt, device="cuda") if k % 3 else None)
        cases.append((host, vs, out, s))
    b = f.batch(items, dots=dots)
    b.launch()
    torch.cuda.synchronize()

    def check(tag):
        for k, (host, vs, out, s) in enumerate(cases):
            x, y, z = vs
            host_of = {id(v.tensor): h for v, h in zip(vs, host)}
            want = oracle_of((x - y) * s + z * 0.75, host_of, dtype, len(host[0]))
            check_bits(out, want, dtype, (tag, k))
            if dots[k] is not None:
                alone = S.salt_dot(x.tensor, y.tensor)
                torch.cuda.synchronize()
                assert dots[k].item() == alone.item(), (tag, k, dots[k].item(), alone.item())

    check("launch")
    g = b.graph()
    for _, _, out, _ in cases:
        out.zero_()
    for d in dots:
        if d is not None:
            d.zero_()
    torch.cuda.synchronize()
    g.launch()
    torch.cuda.synchronize()
    check("graph")


def test_expression_batch_dot_needs_its_first_two_vectors_read_first():
    """A fused dot takes the first two vector arguments; a tree that reads
    another vector first is refused when the plan is made."""
    import torch

    n = 1000
    host = workloads.uniform(n, "f64", 31, 2)
    x, y = (to_dev(h, "f64") for h in host)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    r = torch.empty(1, dtype=torch.float64, device="cuda")
    swapped = expression(lambda a, b: b - a)
    with pytest.raises(S.SaltError):
        swapped.batch([(out, x, y)], dots=[r])
    swapped.batch([(out, x, y)]).launch()          # without the dot it runs
    torch.cuda.synchronize()
    want = oracle.eval_program([T(S.LOAD, 1), T(S.LOAD, 0), T(S.SUB)], host, [], "f64")
    check_bits(out, want, "f64", "swapped")
