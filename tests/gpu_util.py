"""Helpers shared by the GPU tests: moving seeded host inputs to the device
and comparing bit patterns. No arithmetic of the method lives here."""
from __future__ import annotations

import numpy as np

from paper_1109_1264_amd import salt as S

TORCH_DT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16"}
CODE = {"f64": S.F64, "f32": S.F32, "bf16": S.BF16, "f16": S.F16}
BITS = {"f64": np.uint64, "f32": np.uint32, "bf16": np.uint16, "f16": np.uint16}


def to_dev(a: np.ndarray, dtype: str, pad: int = 0, offset: int = 0):
    """Device tensor holding the stored values of ``a``; with ``offset`` the
    tensor is a view starting ``offset`` elements into a larger buffer (so it
    is not 16-byte aligned for odd offsets)."""
    import torch

    tdt = getattr(torch, TORCH_DT[dtype])
    if dtype in ("bf16", "f16"):
        host = torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint16).view(np.int16)).view(tdt)
    else:
        host = torch.from_numpy(np.ascontiguousarray(a))
    buf = torch.empty(len(a) + offset + pad, dtype=tdt, device="cuda")
    t = buf[offset:offset + len(a)]
    t.copy_(host)
    return t


def to_host_bits(t, dtype: str) -> np.ndarray:
    import torch

    c = t.detach().cpu().contiguous()
    if dtype in ("bf16", "f16"):
        return c.view(torch.int16).numpy().view(np.uint16).copy()
    return c.numpy().view(BITS[dtype]).copy()


def empty(n: int, dtype: str, offset: int = 0):
    import torch

    buf = torch.empty(n + offset, dtype=getattr(torch, TORCH_DT[dtype]), device="cuda")
    return buf[offset:offset + n]


def oracle_bits(arr: np.ndarray, dtype: str) -> np.ndarray:
    return np.ascontiguousarray(arr).view(BITS[dtype])


def first_mismatch(got: np.ndarray, want: np.ndarray) -> str:
    bad = np.nonzero(got != want)[0]
    if len(bad) == 0:
        return "none"
    i = bad[0]
    return "%d mismatches, first at %d: got %#x want %#x" % (len(bad), i, int(got[i]), int(want[i]))
