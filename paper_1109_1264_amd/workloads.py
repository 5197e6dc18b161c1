"""Seeded synthetic inputs for the SALT workloads.

This module only draws random inputs. It holds none of the method's
arithmetic, so both the GPU path's tests and the CPU oracle can take their
inputs from it without sharing any evaluation code.

Recipes (the paper measures on synthetic vectors swept across cache and memory
sizes, Sec. 5; no dataset is involved):

- uniform operands: ``numpy.random.Generator(PCG64(seed))``, drawn in operand
  order a, b, c, e, f, g; binary64 as ``2*U[0,1) - 1`` (exact), binary32 as
  ``2*random(float32) - 1`` (exact); 16-bit storage is the binary32 draw
  rounded to the storage type by torch (round-to-nearest-even).
- ``alpha ~ U[0.5, 2)`` from the same generator after the operands.
- ill-conditioned operands for the precision study: random sign, ``log10|x|``
  uniform on [-4, 4], drawn in binary64 and then stored.
- batched lengths: ``round(exp(N(ln 4096, 1.5^2)))`` clipped to [64, 2^20].
- device-side uniform operands for the large sweeps: torch's seeded
  generator on the GPU (Philox), same value recipe, so multi-GiB inputs never
  cross PCIe.
"""
from __future__ import annotations

import math

import numpy as np

DTYPES = ("f64", "f32", "bf16", "f16")
ELEM_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}

# Seeds of the five workload configurations.
SEED_FIG1 = 1109          # d = a + (b - c), FP64, n = 2^20
SEED_SWEEP_BASE = 1264    # BLAS-1 sweep: seed = 1264 + log2(n)
SEED_PRECISION = 3000     # dot / nrm2 at n = 2^26, ill-conditioned
SEED_BATCHED = 4000       # 4096 instances
SEED_SERVED = 5000        # request stream


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _to_storage_bits(x32: np.ndarray, dtype: str) -> np.ndarray:
    """Round binary32 values to a 16-bit storage format (returns uint16 bits)."""
    import torch

    t = torch.from_numpy(np.ascontiguousarray(x32, dtype=np.float32))
    tt = torch.bfloat16 if dtype == "bf16" else torch.float16
    return t.to(tt).view(torch.int16).numpy().view(np.uint16).copy()


def uniform(n: int, dtype: str, seed: int, count: int) -> list[np.ndarray]:
    """``count`` operands of length ``n``, i.i.d. uniform on [-1, 1)."""
    g = _rng(seed)
    out = []
    for _ in range(count):
        if dtype == "f64":
            out.append(2.0 * g.random(n, dtype=np.float64) - 1.0)
        else:
            x = np.float32(2.0) * g.random(n, dtype=np.float32) - np.float32(1.0)
            out.append(x if dtype == "f32" else _to_storage_bits(x, dtype))
    return out


def alpha(seed: int) -> float:
    """alpha ~ U[0.5, 2), from its own stream derived from ``seed``."""
    return float(_rng(seed + 7919).uniform(0.5, 2.0))


def sweep_seed(n: int) -> int:
    return SEED_SWEEP_BASE + int(round(math.log2(n))) if n > 0 else SEED_SWEEP_BASE


def ill_conditioned(n: int, seed: int, count: int = 2) -> list[np.ndarray]:
    """binary64 operands with random sign and log10|x| ~ U[-4, 4]."""
    g = _rng(seed)
    out = []
    for _ in range(count):
        sign = np.where(g.random(n) < 0.5, -1.0, 1.0)
        out.append(sign * np.power(10.0, g.uniform(-4.0, 4.0, n)))
    return out


def store(x64: np.ndarray, dtype: str) -> np.ndarray:
    """Store binary64 values in ``dtype`` (round-to-nearest-even casts)."""
    if dtype == "f64":
        return np.ascontiguousarray(x64, dtype=np.float64)
    x32 = np.ascontiguousarray(x64, dtype=np.float32)
    return x32 if dtype == "f32" else _to_storage_bits(x32, dtype)


def batch_lengths(count: int = 4096, seed: int = SEED_BATCHED, sigma: float = 1.5,
                  median: int = 4096, lo: int = 64, hi: int = 1 << 20) -> np.ndarray:
    """Lognormal instance lengths, clipped."""
    g = _rng(seed)
    n = np.rint(np.exp(g.normal(math.log(median), sigma, count)))
    return np.clip(n, lo, hi).astype(np.int64)


def uniform_device(n: int, dtype: str, seed: int, count: int, device="cuda") -> list:
    """Device-resident uniform [-1, 1) operands from torch's seeded generator."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = []
    for _ in range(count):
        if dtype == "f64":
            t = torch.rand(n, dtype=torch.float64, device=device, generator=g).mul_(2.0).sub_(1.0)
        else:
            t = torch.rand(n, dtype=torch.float32, device=device, generator=g).mul_(2.0).sub_(1.0)
            if dtype == "bf16":
                t = t.to(torch.bfloat16)
            elif dtype == "f16":
                t = t.to(torch.float16)
        out.append(t)
    return out
