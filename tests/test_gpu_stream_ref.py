"""The plain stream reference kernel (bandwidth reference for each
read/write mix): its output is the xor of its inputs, byte for byte, for
every read count, ragged and empty lengths; with no write nothing changes."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1109_1264_amd import salt as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("reads", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("nbytes", [0, 16, 4096 + 48, (1 << 20) + 16 * 37])
def test_output_is_xor_of_inputs(reads, nbytes):
    import torch

    rng = np.random.Generator(np.random.PCG64(reads * 1000 + nbytes % 997))
    host = [rng.integers(0, 256, nbytes + 64, dtype=np.uint8) for _ in range(reads)]
    ins = [torch.from_numpy(h).cuda() for h in host]
    out = torch.full((nbytes + 64,), 0xAB, dtype=torch.uint8, device="cuda")
    S.salt_stream_reference(ins, out, nbytes)
    got = out.cpu().numpy()
    want = host[0][:nbytes].copy()
    for h in host[1:]:
        want ^= h[:nbytes]
    assert np.array_equal(got[:nbytes], want)
    assert (got[nbytes:] == 0xAB).all()              # nothing past `nbytes`
    # reads only: the output is never written
    out2 = torch.full((nbytes + 64,), 0xCD, dtype=torch.uint8, device="cuda")
    S.salt_stream_reference(ins, None, nbytes)
    torch.cuda.synchronize()
    assert (out2.cpu().numpy() == 0xCD).all()
