"""Batched evaluation: many independent items of one tree in one persistent
launch, optionally replayed from a HIP graph (binding of salt_batch_*).

    b = Batch(prog, items, dtype)          # plan + upload of the descriptor table
    b.launch()                             # one persistent launch (+ dot combine)
    g = b.graph(); g.launch()              # the same, captured once, replayed

Each item is a dict with ``n``, ``operands`` (device tensors), ``scalars``,
``out`` (device tensor or None) and ``dot_out`` (one-element device tensor,
float64 for FP64 else float32, or None). Tensors are kept alive by the Batch.
"""
from __future__ import annotations

import ctypes

from . import salt as S


class Graph:
    def __init__(self, handle, owner):
        self._h = handle
        self._owner = owner  # keeps the batch (and its buffers) alive

    def launch(self, stream=None) -> None:
        S.check(S.lib().salt_graph_launch(self._h, S._stream_ptr(stream)))

    def close(self) -> None:
        if self._h:
            S.lib().salt_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    def __init__(self, prog, items, dtype: int, stream=None):
        import torch

        L = S.lib()
        self.dtype = dtype
        self._keep = []
        arr = (S.BatchItem * max(1, len(items)))()
        for i, it in enumerate(items):
            b = arr[i]
            b.n = int(it["n"])
            for k, t in enumerate(it.get("operands", [])):
                if t is not None:
                    if S.dtype_code(t) != dtype:
                        raise TypeError("operand dtype differs from the batch dtype")
                    if t.numel() < b.n:
                        raise ValueError("operand shorter than n")
                    b.operands[k] = S._dev(t)
                    self._keep.append(t)
            for j, v in enumerate(it.get("scalars", [])):
                b.scalars[j] = float(v)
            out = it.get("out")
            if out is not None:
                if S.dtype_code(out) != dtype or out.numel() < b.n:
                    raise ValueError("bad output tensor")
                b.out = S._dev(out)
                self._keep.append(out)
            dot = it.get("dot_out")
            if dot is not None:
                want = torch.float64 if dtype == S.F64 else torch.float32
                if dot.dtype != want or not dot.is_cuda:
                    raise TypeError("dot_out must be a %s device tensor" % want)
                b.dot_out = dot.data_ptr()
                self._keep.append(dot)
        parr, plen = S._prog(prog)
        nops = 1 + max([t >> 8 for t in prog if t & 0xFF == S.LOAD], default=-1)
        nsc = 1 + max([t >> 8 for t in prog if t & 0xFF == S.SCALAR], default=-1)
        h = ctypes.c_void_p()
        S.check(L.salt_batch_plan_create(parr, plen, max(nops, 0), max(nsc, 0), arr, len(items), dtype,
                                         ctypes.byref(h)))
        self._plan = h
        tb, wb, tiles = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int64()
        S.check(L.salt_batch_plan_info(h, ctypes.byref(tb), ctypes.byref(wb), ctypes.byref(tiles)))
        self.table_bytes, self.ws_bytes, self.tiles = tb.value, wb.value, tiles.value
        dev = "cuda"
        # torch's allocator hands out at least 512-byte aligned blocks
        self.table = torch.empty(max(256, self.table_bytes), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(max(1, (self.ws_bytes + 7) // 8), dtype=torch.float64, device=dev)
        S.check(L.salt_batch_upload(h, self.table.data_ptr(), self.table.numel(), S._stream_ptr(stream)))

    def launch(self, stream=None, config=None) -> None:
        S.check(S.lib().salt_batch_launch(self._plan, self.ws.data_ptr(), self.ws.numel() * 8,
                                          S._stream_ptr(stream), S._cfg(config)))

    def graph(self, config=None) -> Graph:
        g = ctypes.c_void_p()
        S.check(S.lib().salt_batch_graph_create(self._plan, self.ws.data_ptr(), self.ws.numel() * 8,
                                                S._cfg(config), ctypes.byref(g)))
        return Graph(g, self)

    def close(self) -> None:
        if getattr(self, "_plan", None):
            S.lib().salt_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
