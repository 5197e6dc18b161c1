"""Host-side checks of the serving trace builder (no GPU): a request longer
than its element type's pool is refused instead of pointing past the pool,
and the serving workload's trace covers every (tree, element type) pair."""
from __future__ import annotations

import pytest

from paper_1109_1264_amd import serve as V


class FakePool:
    """Element counts and addresses only; nothing is allocated."""

    def __init__(self, total_bytes, mix=V.MIX):
        self.n = {d: int(total_bytes * f) // {"f64": 8, "f32": 4, "bf16": 2}[d] // 4096 * 4096 for d, f in mix}

    def elems(self, dt):
        return self.n[dt]

    def ptr(self, dt, off):
        return 1 << 40 | off


def test_request_longer_than_pool_is_refused():
    pool = FakePool(1 << 20)                      # 32768 binary64 elements
    with pytest.raises(ValueError):
        V.make_trace(pool, 50, seed=1, rate=None, lo=16, hi=17, mix=(("f64", 1.0),))


def test_operand_ranges_stay_inside_the_pool():
    pool = FakePool(6 << 30)
    es = {"f64": 8, "f32": 4, "bf16": 2}
    trace, meta = V.make_trace(pool, 600, seed=5010, rate=60000.0, lo=8, hi=24)
    for r, (tree, dt, n, offs, alpha) in zip(trace, meta):
        assert len(offs) == V.tree_loads(tree)
        for k, o in enumerate(offs):
            assert 0 <= o and o + n <= pool.elems(dt) and o % 64 == 0
            assert r.operands[k] == pool.ptr(dt, o)
        assert 0.5 <= alpha < 2.0


def test_serving_workload_trace_covers_every_tree_and_type():
    """The trace of the GPU test at the serving workload's shapes: all 15
    (tree, type) pairs, lengths reaching the top octave below 2^24."""
    pool = FakePool(6 << 30)
    _, meta = V.make_trace(pool, 600, seed=5010, rate=60000.0, lo=8, hi=24)
    assert {(m[0], m[1]) for m in meta} == {(t, d) for t in V.TREES for d in ("f32", "bf16", "f64")}
    assert max(m[2] for m in meta) > (1 << 23)
    assert max(m[2] for m in meta) <= (1 << 24)
    total = sum(m[2] for m in meta)
    print("elements", total)
