"""The tuner's host logic on the CPU: the candidate grid, the buffer-rotation
policy of the streaming regime, and a table it writes being read back by the
library (kind names, routes, nearest-size lookup). No kernel runs."""
from __future__ import annotations

from paper_1109_1264_amd import autotune as A
from paper_1109_1264_amd import salt as S


def test_candidate_grid():
    c = A.candidates("eval", 1 << 20, S.F64, 256)
    assert len(c) == 4 * 2 * 6 and len(set(c)) == len(c)
    assert {u for u, _, _ in c} == {1, 2, 4, 8}
    assert {b for _, _, b in c} == {0, 256, 512, 1024, 2048, 4096}
    assert {u for u, _, _ in A.candidates("dot", 1 << 20, S.F32, 256)} == {2, 4, 8, 16}
    assert {u for u, _, _ in A.candidates("batch", 1 << 20, S.F32, 256)} == {2, 4, 8}


def workload(arrays, dtype, n_max, rotate, rotate_from=4 << 20):
    w = A.Workload.__new__(A.Workload)   # no device buffers: only the policy
    w.arrays, w.dtype, w.n_max, w.rotate, w.rotate_from = arrays, dtype, n_max, rotate, rotate_from
    return w


def test_rotation_policy():
    # default: cache-resident, never rotated
    assert workload(4, S.F64, 1 << 27, False).sets(1 << 20) == 1
    w = workload(4, S.F64, 1 << 27, True)
    assert w.sets(1 << 16) == 1            # 2 MiB working set: below 4 MiB
    assert w.sets(1 << 20) == 32           # 32 MiB: 1 GiB worth of slices
    assert w.sets(1 << 24) == 2            # 512 MiB
    assert w.sets(1 << 25) == 1            # 1 GiB: streams anyway
    assert workload(2, S.F32, 1 << 28, True).sets(1 << 19) == 64   # capped
    # never more slices than the buffers hold
    assert workload(4, S.F32, 1 << 22, True).sets(1 << 20) == 4
    for n in (1 << 18, 1 << 20, 1 << 22):
        w = workload(3, S.BF16, 1 << 29, True)
        assert w.sets(n) * n <= w.n_max


def test_rotation_threshold():
    """Streaming only from the threshold up: below it the working set is
    timed cache-resident."""
    w = workload(2, S.F32, 1 << 28, True, rotate_from=128 << 20)
    assert w.sets(1 << 23) == 1            # 64 MiB: resident
    assert w.sets(1 << 24) == 8            # 128 MiB: 1 GiB worth of slices
    assert w.sets(1 << 26) == 2            # 512 MiB
    assert w.sets(1 << 27) == 1            # 1 GiB


def test_reduction_pairs_follow_the_library_catalogue():
    """The tuner's pair list is the library's reduction-pair catalogue, in
    order (each routes to its own index)."""
    for i, (px, py) in enumerate(A.PAIRS):
        assert S.salt_reduce_expr_route(px, py, 2, 1) == i


def test_written_table_reads_back(tmp_path):
    rows = [("eval", 2, S.F64, 20, 2, 1, 512, 0.0043, 7892.0),
            ("dot", -1, S.F32, 26, 16, 0, 1024, 0.085, 6300.0),
            ("nrm2", -2, S.BF16, 24, 4, 1, 0, 0.019, 3500.0),
            ("batch", 5, S.F32, 25, 8, 1, 4096, 0.153, 5300.0),
            ("dot", A.PAIR_ROUTE0, S.BF16, 28, 8, 1, 256, 0.171, 6266.0)]
    p = tmp_path / "t.txt"
    A.write_table(rows, str(p))
    S.salt_tuning_load(str(p))
    try:
        assert S.salt_tuning_lookup(0, 2, S.F64, 1 << 20) == (2, 1, 512)
        assert S.salt_tuning_lookup(1, -1, S.F32, 1 << 26) == (16, 0, 1024)
        assert S.salt_tuning_lookup(2, -2, S.BF16, 1 << 24) == (4, 1, 0)
        assert S.salt_tuning_lookup(3, 5, S.F32, 50645917) == (8, 1, 4096)
        assert S.salt_tuning_lookup(1, A.PAIR_ROUTE0, S.BF16, 1 << 28) == (8, 1, 256)
    finally:
        S.salt_tuning_load(None)


def test_tuned_interpreter_programs_stay_on_the_interpreter():
    """The expression-reduction pair tuned under route -2 is not one with an
    ahead-of-time kernel, and the eval program tuned under routes -1 and -3
    is not a catalogue tree."""
    assert S.salt_reduce_expr_route(A.EXPR_P, A.EXPR_Q, 2, 0) == -1
    assert S.salt_reduce_expr_route(A.EXPR_P, None, 2, 0) == -1
    assert S.salt_program_route(A.INTERP_PROG, 3, 0) == -1


def test_compiled_pair_kinds_and_merge(tmp_path):
    """The compiled expression reductions are tuned under route -3 with the
    interpreter's candidate unrolls, and a merged run replaces only the
    (kind, route, dtype) groups it tunes."""
    assert {u for u, _, _ in A.candidates("dotj", 1 << 20, S.F32, 256)} == {2, 4, 8}
    assert {u for u, _, _ in A.candidates("nrm2j", 1 << 20, S.F32, 256)} == {2, 4, 8}
    old = [("dot", -2, S.F32, 20, 4, 1, 0, 0.01, 100.0),
           ("dot", A.JIT_ROUTE, S.F32, 20, 2, 0, 0, 0.02, 50.0),
           ("dot", A.JIT_ROUTE, S.F64, 20, 2, 0, 0, 0.02, 50.0)]
    p = tmp_path / "t.txt"
    A.write_table(old, str(p))
    back = A.read_table(str(p))
    assert [r[:7] for r in back] == [r[:7] for r in old]
    assert abs(back[0][7] - 0.01) < 1e-9 and back[0][8] == 100.0
    new = [("dot", A.JIT_ROUTE, S.F32, 20, 8, 1, 512, 0.01, 90.0),
           ("dot", A.JIT_ROUTE, S.F32, 22, 8, 1, 512, 0.03, 95.0)]
    m = A.merged(back, new)
    assert [r[:7] for r in m] == [r[:7] for r in (old[0], old[2], new[0], new[1])]
