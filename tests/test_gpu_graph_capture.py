"""The library's calls inside a captured HIP graph (torch.cuda.graph): a tree
evaluation, axpy, dot, nrm2, asum and iamax captured once and replayed
several times, with eager work that changes the inputs between replays; every
replay must give the bits the same calls give eagerly on the same inputs
(no call may record work a replay would get wrong, such as a memset)."""
from __future__ import annotations

import pytest

from paper_1109_1264_amd import salt as S
from paper_1109_1264_amd import workloads

pytestmark = pytest.mark.gpu

T = S.token
FIG1 = [T(S.LOAD, 0), T(S.LOAD, 1), T(S.LOAD, 2), T(S.SUB), T(S.ADD)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_replays_match_eager(dtype):
    import torch

    n = 3 * S.salt_reduce_tile_elems(S.F64 if dtype == "f64" else S.F32) + 123
    a, b, c = workloads.uniform_device(n, dtype, 6100, 3)
    d = torch.empty_like(a)
    y = torch.empty_like(a)
    code = S.F64 if dtype == "f64" else S.F32
    rdt = torch.float64 if dtype == "f64" else torch.float32
    ws = S.workspace(n, code)
    r_dot, r_nrm, r_asum = (torch.empty(1, dtype=rdt, device="cuda") for _ in range(3))
    r_max = torch.empty(1, dtype=torch.int64, device="cuda")

    def calls():
        S.salt_eval(FIG1, [a, b, c], [], d)
        y.copy_(c)
        S.salt_axpy(0.75, a, y)
        S.salt_dot(a, d, result=r_dot, ws=ws)
        S.salt_nrm2(y, result=r_nrm, ws=ws)
        S.salt_asum(b, result=r_asum, ws=ws)
        S.salt_iamax(d, result=r_max, ws=ws)

    def snapshot():
        torch.cuda.synchronize()
        return [t.clone() for t in (d, y, r_dot, r_nrm, r_asum, r_max)]

    calls()
    snapshot()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calls()
    for k in range(4):
        # eager work between replays: new inputs
        a.mul_(1.5).sub_(0.25)
        b.add_(0.125 * (k + 1))
        torch.cuda.synchronize()
        g.replay()
        got = snapshot()
        calls()
        want = snapshot()
        for i, (x, w) in enumerate(zip(got, want)):
            assert torch.equal(x.view(torch.uint8), w.view(torch.uint8)), (dtype, k, i)
    del g
