"""Serving: a request stream of expression evaluations over operands resident
in device memory, run by libsalt's native loop (salt_serve_trace).

This module builds the resident operand pool and request traces (Poisson
arrivals over five trees, log-uniform lengths, a dtype mix), calls the C loop,
and summarises latency (arrival -> GPU completion) and throughput.

Trees served (all within 2-6 operands, depth <= 4, ops add/sub/mul/scale):
    T1 fig1   d = a + (b - c)
    T2 axpy   d = alpha*x + y
    T3 tree5  d = a*b + c*e - f
    T4 t4     d = alpha*(a + b) - c*e
    T5 t5     d = ((a*b + c)*(e - f)) + alpha*g
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import salt as S

TREES = ("fig1", "axpy", "tree5", "t4", "t5")
MIX = (("f32", 0.5), ("bf16", 0.3), ("f64", 0.2))
DT = {"f64": S.F64, "f32": S.F32, "bf16": S.BF16, "f16": S.F16}


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("table_arena", ctypes.c_void_p), ("table_bytes", ctypes.c_size_t),
                ("max_inflight", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("release_on_complete", ctypes.c_int32), ("grouping", ctypes.c_int32),
                ("launch", ctypes.POINTER(S.LaunchConfig)), ("range_bytes", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("tree", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("n", ctypes.c_int64), ("operands", ctypes.c_void_p * S.MAX_OPERANDS),
                ("scalars", ctypes.c_double * S.MAX_SCALARS)]


class RequestResult(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("launch_s", ctypes.c_double), ("complete_s", ctypes.c_double),
                ("out", ctypes.c_void_p), ("status", ctypes.c_int32), ("batch", ctypes.c_int32)]


def _declare():
    L = S.lib()
    if not getattr(L, "_serve_declared", False):
        L.salt_serve_trace.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(Request), ctypes.c_int32,
                                       ctypes.POINTER(RequestResult)]
        L.salt_serve_trace.restype = ctypes.c_int32
        L._serve_declared = True
    return L


def catalogue_ids():
    names = [n for n, _ in S.salt_catalogue()]
    return {t: names.index(t) for t in TREES}


def tree_loads(name: str) -> int:
    prog = dict(S.salt_catalogue())[name]
    return 1 + max(t >> 8 for t in prog if t & 0xFF == S.LOAD)


class Pool:
    """Device-resident operand pool, one flat buffer per element type, filled
    once from torch's seeded generator with uniform [-1, 1) values and never
    written again (served requests always write fresh outputs)."""

    def __init__(self, total_bytes: int, seed: int, mix=MIX, device="cuda"):
        import torch

        self.buf = {}
        g = torch.Generator(device=device)
        g.manual_seed(seed)
        for name, frac in mix:
            es = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[name]
            n = int(total_bytes * frac) // es // 4096 * 4096
            t = torch.empty(n, dtype={"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
                                      "f16": torch.float16}[name], device=device)
            chunk = 1 << 26
            for s in range(0, n, chunk):
                e = min(n, s + chunk)
                t[s:e] = torch.rand(e - s, generator=g, device=device, dtype=torch.float32).mul_(2).sub_(1)
            self.buf[name] = t

    def elems(self, dtype: str) -> int:
        return self.buf[dtype].numel()

    def ptr(self, dtype: str, offset: int) -> int:
        t = self.buf[dtype]
        return t.data_ptr() + offset * t.element_size()


def make_trace(pool: Pool, count: int, seed: int, rate: float | None, lo: int = 8, hi: int = 24,
               mix=MIX, trees=TREES, fp64_only: bool = False):
    """Requests with Poisson arrivals at ``rate`` per second (None: all at
    t = 0), uniform tree choice, n = round(2^U[lo, hi]), dtype by ``mix``
    (or all binary64), operands at random 64-element-aligned offsets."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ids = catalogue_ids()
    names = [m[0] for m in mix]
    probs = np.array([m[1] for m in mix], dtype=np.float64)
    probs /= probs.sum()
    arr = (Request * count)()
    t = 0.0
    meta = []
    for i in range(count):
        if rate:
            t += rng.exponential(1.0 / rate)
        tree = trees[int(rng.integers(len(trees)))]
        dt = "f64" if fp64_only else names[int(rng.choice(len(names), p=probs))]
        n = int(round(2.0 ** rng.uniform(lo, hi)))
        r = arr[i]
        r.arrival_s = t
        r.tree = ids[tree]
        r.dtype = DT[dt]
        r.n = n
        if n > pool.elems(dt):
            raise ValueError("request length %d exceeds the %s pool (%d elements)" % (n, dt, pool.elems(dt)))
        span = pool.elems(dt) - n
        offs = []
        for k in range(tree_loads(tree)):
            off = int(rng.integers(0, max(1, span // 64))) * 64
            r.operands[k] = pool.ptr(dt, off)
            offs.append(off)
        r.scalars[0] = float(rng.uniform(0.5, 2.0))
        meta.append((tree, dt, n, offs, r.scalars[0]))
    return arr, meta


def request_host_bits(pool: Pool, arena, r, m, idx=None):
    """Host copies of one served request: its operand values and its output
    at element indices ``idx`` (all elements when None), as numpy arrays of
    the storage type (16-bit types as uint16 bit patterns). The output is read
    from the arena, so the request must have been served with kept outputs."""
    import torch

    tree, dt, n, offs, _ = m
    src = pool.buf[dt]
    es = src.element_size()
    off = (r.out - arena.data_ptr()) // es
    if (r.out - arena.data_ptr()) % es:
        raise ValueError("output not aligned to its element size")
    out_view = arena.view(src.dtype)[off:off + n]
    ti = None if idx is None else torch.as_tensor(np.asarray(idx, dtype=np.int64), device=src.device)

    def host(t):
        t = t if ti is None else t.index_select(0, ti)
        t = t.cpu()
        if dt in ("bf16", "f16"):
            return t.view(torch.int16).numpy().view(np.uint16).copy()
        return t.numpy().copy()
    ops = [host(src[o:o + n]) for o in offs]
    return ops, host(out_view)


GROUP_MIXED, GROUP_BY_TREE, GROUP_AUTO = 0, 1, 2


def serve(trace, arena, table, max_inflight=4096, n_streams=4, max_batch=512, depth=2, keep_outputs=False,
          grouping=GROUP_MIXED, launch=None, range_bytes=0):
    """Run the trace through the native loop; returns the results array.
    Per element type a batch runs one mixed-tree launch (GROUP_MIXED), one
    single-tree launch per tree (GROUP_BY_TREE), or the latter only when the
    type's requests hold at least 2^26 elements (GROUP_AUTO). ``launch``:
    (unroll, nontemporal, blocks) for every batched launch (0 / -1 / -1
    keep the tuned value), or None: tuned. ``range_bytes``: bytes per
    operand of one launch of a long tile list (0: the library's 256 MiB,
    -1: never split)."""
    L = _declare()
    count = len(trace)
    res = (RequestResult * max(1, count))()
    knobs = S.LaunchConfig(*launch) if launch is not None else None
    cfg = ServerConfig(arena.data_ptr(), arena.numel() * arena.element_size(), table.data_ptr(),
                       table.numel() * table.element_size(), max_inflight, n_streams, max_batch, depth,
                       0 if keep_outputs else 1, grouping,
                       ctypes.pointer(knobs) if knobs is not None else None, range_bytes)
    S.check(L.salt_serve_trace(ctypes.byref(cfg), trace, count, res))
    return res


def request_bytes(meta) -> np.ndarray:
    es = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
    return np.array([(tree_loads(m[0]) + 1) * m[2] * es[m[1]] for m in meta], dtype=np.float64)


def summarize(res, meta) -> dict:
    st = np.array([r.status for r in res])
    ok = st == 0
    arr = np.array([r.arrival_s for r in res])[ok]
    com = np.array([r.complete_s for r in res])[ok]
    lat = (com - arr) * 1e3
    span = float(com.max() - arr.min()) if ok.any() else float("nan")
    nbytes = float(request_bytes(meta)[ok].sum())
    batches = len({r.batch for r, o in zip(res, ok) if o})
    return {"requests": int(ok.sum()), "rejected": int((~ok).sum()),
            "p50_ms": round(float(np.percentile(lat, 50)), 4) if ok.any() else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 4) if ok.any() else None,
            "mean_ms": round(float(lat.mean()), 4) if ok.any() else None,
            "throughput_rps": round(ok.sum() / span, 1) if span > 0 else None,
            "GBps": round(nbytes / span / 1e9, 1) if span > 0 else None,
            "makespan_s": round(span, 4), "batches": batches}


def default_buffers(arena_bytes: int = 8 << 30, table_bytes: int = 64 << 20):
    import torch

    arena = torch.empty(arena_bytes // 8, dtype=torch.float64, device="cuda")
    table = torch.empty(table_bytes // 8, dtype=torch.float64, device="cuda")
    return arena, table
