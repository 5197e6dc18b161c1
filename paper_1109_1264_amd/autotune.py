"""Measured choice of launch knobs (unroll, non-temporal hints, grid size).

The paper picks the number of instruction packages per loop by trial, few for
small vectors and many for large ones (Sec. 4.3). Here every candidate
(unroll x non-temporal x grid) is timed with HIP events on the launch stream
for each (kind, tree, element type, size) and the fastest one is written to
a tuning table that libsalt loads at start-up (``salt_tuning.txt`` beside the
library, or ``$SALT_TUNE_FILE``). None of the knobs changes a result bit, so
the table only moves time.

    python -m paper_1109_1264_amd.autotune --rotate --rotate-from-mib 128 \
        --out paper_1109_1264_amd/salt_tuning.txt
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

from . import salt as S

KIND = {"eval": 0, "dot": 1, "nrm2": 2}
DT_NAMES = {"f64": S.F64, "f32": S.F32, "bf16": S.BF16, "f16": S.F16}


def _torch_dtype(d):
    import torch

    return {S.F64: torch.float64, S.F32: torch.float32, S.BF16: torch.bfloat16, S.F16: torch.float16}[d]


def candidates(kind: str, n: int, dtype: int, cus: int):
    unrolls = {"eval": (1, 2, 4, 8), "interp": (1, 2, 4), "jit": (1, 2, 4), "batch": (2, 4, 8),
               "dotx": (2, 4, 8), "nrm2x": (2, 4, 8), "dotj": (2, 4, 8), "nrm2j": (2, 4, 8)}.get(kind, (2, 4, 8, 16))
    grids = [0] + [cus * k for k in (1, 2, 4, 8, 16)]
    out = []
    for u in unrolls:
        for nt in (0, 1):
            for b in grids:
                out.append((u, nt, b))
    return out


def time_config(fn, cfg, reps: int, warm: int = 2) -> float:
    """Device time (ms) per launch of fn(cfg): `reps` launches captured in one
    HIP graph, replayed three times between two events, median. Back-to-back
    launches without Python or host launch overhead, which at small sizes
    would otherwise hide the device time the knobs change."""
    import torch

    for _ in range(warm):
        fn(cfg)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn(cfg)
    g.replay()
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) / reps)
    del g
    return sorted(ts)[1]


# Representative programs outside the catalogue: they run on the interpreter
# (eval, route -1), on their run-time compiled kernel (eval, route -3), on
# the interpreted expression reductions (dot / nrm2, route -2) and on the
# expression reductions' run-time compiled kernels (dot / nrm2, route -3).
T_ = S.token
INTERP_PROG = [T_(S.LOAD, 0), T_(S.LOAD, 1), T_(S.ADD), T_(S.LOAD, 2), T_(S.MUL)]   # (a + b) * c
# interpreted expression reductions: a pair outside the reduction catalogue
EXPR_P = [T_(S.LOAD, 0), T_(S.LOAD, 1), T_(S.MUL)]                                  # a * b
EXPR_Q = [T_(S.LOAD, 0), T_(S.LOAD, 1), T_(S.ADD)]                                  # a + b
# The reduction pairs with ahead-of-time kernels (route -16 - index), in the
# library's catalogue order: (P, Q or None for nrm2).
_SUM, _DIFF = [T_(S.LOAD, 0), T_(S.LOAD, 1), T_(S.ADD)], [T_(S.LOAD, 0), T_(S.LOAD, 1), T_(S.SUB)]
PAIRS = [(_SUM, _DIFF),                                                            # dot(a + b, a - b)
         (_DIFF, None),                                                            # nrm2(a - b)
         ([T_(S.SCALAR, 0), T_(S.LOAD, 0), T_(S.MUL), T_(S.LOAD, 1), T_(S.ADD)], None)]  # nrm2(alpha*a + b)
PAIR_ROUTE0 = -16
JIT_ROUTE = -3   # trees outside the catalogue on their run-time compiled kernels


class Workload:
    """Device buffers for one (kind, tree, dtype) at the largest size swept."""

    def __init__(self, kind: str, tree: str | None, dtype: int, n_max: int, rotate: bool = False,
                 rotate_from: int = 4 << 20):
        import torch

        if rotate:
            # at least 1 GiB per buffer, so that sizes below it have disjoint
            # slices to rotate through (see sets())
            n_max = max(n_max, (1 << 30) // S.ELEM_BYTES[dtype])
        self.kind, self.dtype, self.n_max, self.rotate = kind, dtype, n_max, rotate
        self.rotate_from = rotate_from
        td = _torch_dtype(dtype)
        cat = dict(S.salt_catalogue())
        self.route = -1
        if kind in ("interp", "jit"):
            self.prog = INTERP_PROG
            self.route = -1 if kind == "interp" else JIT_ROUTE
            self.ops = [torch.rand(n_max, device="cuda").to(td) for _ in range(3)]
            self.sc = []
            self.out = torch.empty(n_max, dtype=td, device="cuda")
            self.arrays = 4
        elif kind.startswith("pair"):
            self.pair = int(kind[4:])
            self.route = PAIR_ROUTE0 - self.pair
            self.ops = [torch.rand(n_max, device="cuda").to(td) for _ in range(2)]
            self.ws = S.workspace(n_max, dtype)
            self.res = torch.empty(1, dtype=torch.float64 if dtype == S.F64 else torch.float32, device="cuda")
            self.arrays = 2
        elif kind in ("dotx", "nrm2x", "dotj", "nrm2j"):
            # the same pair on the interpreter (route -2) or on its run-time
            # compiled kernel (JIT_ROUTE)
            self.route = -2 if kind.endswith("x") else JIT_ROUTE
            self.ops = [torch.rand(n_max, device="cuda").to(td) for _ in range(2)]
            self.ws = S.workspace(n_max, dtype)
            self.res = torch.empty(1, dtype=torch.float64 if dtype == S.F64 else torch.float32, device="cuda")
            self.arrays = 2
        elif kind == "eval":
            self.prog = cat[tree]
            self.route = [name for name, _ in S.salt_catalogue()].index(tree)
            nops = 1 + max([t >> 8 for t in self.prog if t & 0xFF == S.LOAD], default=-1)
            nsc = 1 + max([t >> 8 for t in self.prog if t & 0xFF == S.SCALAR], default=-1)
            self.ops = [torch.rand(n_max, device="cuda").to(td) for _ in range(max(nops, 1))][:nops]
            self.sc = [1.25] * nsc
            self.out = torch.empty(n_max, dtype=td, device="cuda")
            self.arrays = nops + 1
        else:
            self.x = torch.rand(n_max, device="cuda").to(td)
            self.y = torch.rand(n_max, device="cuda").to(td) if kind == "dot" else self.x
            self.ws = S.workspace(n_max, dtype)
            self.res = torch.empty(1, dtype=torch.float64 if dtype == S.F64 else torch.float32, device="cuda")
            self.arrays = 2 if kind == "dot" else 1

    def sets(self, n: int) -> int:
        """Disjoint slices of the buffers that launches at size n cycle
        through. Without rotation (the default) every launch reuses the same
        buffers, so working sets below the 256 MiB last-level cache are timed
        cache-resident, as in iterative use of the same vectors. With
        rotation: enough slices for about 1 GiB (at most 64), so a working
        set between `rotate_from` (4 MiB by default) and 1 GiB streams from
        HBM."""
        ws = self.arrays * S.ELEM_BYTES[self.dtype] * n
        if not self.rotate or ws >= (1 << 30) or ws < max(4 << 20, self.rotate_from):
            return 1
        return int(min(64, self.n_max // n, -(-(1 << 30) // ws)))

    def fn(self, n: int):
        sets, state = self.sets(n), {"k": 0}

        def sl(t):
            k = state["k"] % sets
            return t[k * n:(k + 1) * n]

        def step(call):
            def run(cfg):
                call(cfg)
                state["k"] += 1
            return run

        if self.kind.startswith("pair"):
            px, py = PAIRS[self.pair]
            if py is None:
                return step(lambda cfg: S.salt_nrm2_expr(px, [sl(o) for o in self.ops], [1.25], n=n,
                                                         result=self.res, ws=self.ws, config=cfg))
            return step(lambda cfg: S.salt_dot_expr(px, py, [sl(o) for o in self.ops], [1.25], n=n,
                                                    result=self.res, ws=self.ws, config=cfg))
        if self.kind in ("dotx", "dotj"):
            return step(lambda cfg: S.salt_dot_expr(EXPR_P, EXPR_Q, [sl(o) for o in self.ops], [], n=n,
                                                    result=self.res, ws=self.ws, config=cfg))
        if self.kind in ("nrm2x", "nrm2j"):
            return step(lambda cfg: S.salt_nrm2_expr(EXPR_P, [sl(o) for o in self.ops], [], n=n, result=self.res,
                                                     ws=self.ws, config=cfg))
        if self.kind in ("eval", "interp", "jit"):
            return step(lambda cfg: S.salt_eval(self.prog, [sl(o) for o in self.ops], self.sc, sl(self.out),
                                                config=cfg))
        if self.kind == "dot":
            return step(lambda cfg: S.salt_dot(sl(self.x), sl(self.y), result=self.res, ws=self.ws, config=cfg))
        return step(lambda cfg: S.salt_nrm2(sl(self.x), result=self.res, ws=self.ws, config=cfg))


def tune(kind: str, tree: str | None, dtype: int, log2ns, reps: int = 10, verbose: bool = False,
         rotate: bool = False, rotate_from: int = 4 << 20):
    """Rows (kind, route, dtype, log2n, unroll, nt, blocks, best_ms, GBps)."""
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    w = Workload(kind, tree, dtype, 1 << max(log2ns), rotate=rotate, rotate_from=rotate_from)
    # the interpreter's rows are timed on the interpreter, the compiled
    # trees' rows on the compiled kernel
    if kind in ("interp", "dotx", "nrm2x"):
        S.salt_jit_set_mode(S.JIT_OFF)
    elif kind == "jit":
        S.salt_jit_set_mode(S.JIT_EXPLICIT)
        S.salt_jit_compile(w.prog, len(w.ops), 0, dtype)
    elif kind in ("dotj", "nrm2j"):
        S.salt_jit_set_mode(S.JIT_EXPLICIT)
        S.salt_jit_compile_reduce(EXPR_P, EXPR_Q if kind == "dotj" else None, 2, 0, dtype)
    rows = []
    for l in log2ns:
        n = 1 << l
        fn = w.fn(n)
        reps_l = max(reps if l >= 20 else reps * 3, w.sets(n))
        best = None
        for cfg in candidates(kind, n, dtype, cus):
            t = time_config(fn, cfg, reps_l)
            if best is None or t < best[0]:
                best = (t, cfg)
        t, (u, nt, b) = best
        gbps = w.arrays * n * S.ELEM_BYTES[dtype] / (t * 1e-3) / 1e9
        table_kind = {"interp": "eval", "jit": "eval", "dotx": "dot", "nrm2x": "nrm2", "dotj": "dot",
                      "nrm2j": "nrm2"}.get(kind, kind)
        if kind.startswith("pair"):
            table_kind = "nrm2" if PAIRS[w.pair][1] is None else "dot"
        rows.append((table_kind, w.route, dtype, l, u, nt, b, t, gbps))
        if verbose:
            print("tuned %s %s %s 2^%d: unroll=%d nt=%d blocks=%d %.4f ms %.0f GB/s"
                  % (kind, tree or "", S.DTYPE_NAMES[dtype], l, u, nt, b, t, gbps), file=sys.stderr, flush=True)
    S.salt_jit_set_mode(S.JIT_AUTO)
    return rows


class BatchWorkload:
    """A batched launch of one catalogue tree (or, for tree "compiled", of
    the representative tree outside the catalogue, whose batched kernels are
    compiled at plan creation) over items of the given lengths (operands
    carved from flat device buffers at 64-element boundaries)."""

    def __init__(self, tree: str, dtype: int, lengths, with_dot: bool, seed: int = 1):
        import numpy as np
        import torch

        from .batch import Batch

        td = _torch_dtype(dtype)
        if tree == "compiled":
            prog, self.route = INTERP_PROG, JIT_ROUTE
        else:
            prog = dict(S.salt_catalogue())[tree]
            self.route = [name for name, _ in S.salt_catalogue()].index(tree)
        nops = 1 + max([t >> 8 for t in prog if t & 0xFF == S.LOAD], default=-1)
        offs = np.zeros(len(lengths) + 1, dtype=np.int64)
        offs[1:] = np.cumsum((np.asarray(lengths) + 63) // 64 * 64)
        cap = int(offs[-1])
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        self.bufs = [torch.rand(cap, device="cuda", generator=g).to(td) for _ in range(nops)]
        self.out = torch.empty(cap, dtype=td, device="cuda")
        self.dots = torch.empty(len(lengths), dtype=torch.float64 if dtype == S.F64 else torch.float32,
                                device="cuda")
        items = []
        for k, n in enumerate(lengths):
            a, b = int(offs[k]), int(offs[k]) + int(n)
            items.append({"n": int(n), "operands": [t[a:b] for t in self.bufs], "scalars": [1.25],
                          "out": self.out[a:b], "dot_out": self.dots[k:k + 1] if with_dot else None})
        self.batch = Batch(prog, items, dtype)
        self.total = int(np.sum(lengths))
        self.arrays = nops + 1

    def fn(self):
        return lambda cfg: self.batch.launch(config=cfg)


def tune_batch(tree: str, dtype: int, scenarios, with_dot: bool, reps: int = 10, verbose: bool = False):
    """One row per scenario (a list of item lengths), keyed by log2 of the
    total number of elements."""
    import math

    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    rows = []
    for lengths in scenarios:
        w = BatchWorkload(tree, dtype, lengths, with_dot)
        fn = w.fn()
        best = None
        for cfg in candidates("batch", w.total, dtype, cus):
            t = time_config(fn, cfg, reps)
            if best is None or t < best[0]:
                best = (t, cfg)
        t, (u, nt, b) = best
        l = int(math.log2(max(1, w.total)))
        gbps = w.arrays * w.total * S.ELEM_BYTES[dtype] / (t * 1e-3) / 1e9
        rows.append(("batch", w.route, dtype, l, u, nt, b, t, gbps))
        if verbose:
            print("tuned batch %s %s %d items 2^%d elems: unroll=%d nt=%d blocks=%d %.4f ms %.0f GB/s"
                  % (tree, S.DTYPE_NAMES[dtype], len(lengths), l, u, nt, b, t, gbps), file=sys.stderr, flush=True)
        del w
        torch.cuda.empty_cache()
    return rows


def serving_scenarios(seed: int = 11):
    """Item-length mixes like the served batches: log-uniform 2^8..2^24."""
    import numpy as np

    rng = np.random.Generator(np.random.PCG64(seed))
    return [np.rint(2.0 ** rng.uniform(8, 24, k)).astype(np.int64) for k in (4, 16, 64, 256)]


def read_table(path: str):
    """Rows of a tuning table, in write_table's tuple form (the ms and GB/s
    comment figures are 0 where a row has none)."""
    rows = []
    with open(path) as fh:
        for line in fh:
            body, _, note = line.partition("#")
            f = body.split()
            if len(f) != 7:
                continue
            m = re.match(r"\s*([0-9.]+) ms ([0-9.]+) GB/s", note)
            t, g = (float(m.group(1)), float(m.group(2))) if m else (0.0, 0.0)
            rows.append((f[0], int(f[1]), int(f[2]), int(f[3]), int(f[4]), int(f[5]), int(f[6]), t, g))
    return rows


def merged(old, new):
    """old's rows, with every (kind, route, dtype) that new tunes replaced by
    new's rows; new rows come last."""
    keys = {(r[0], r[1], r[2]) for r in new}
    return [r for r in old if (r[0], r[1], r[2]) not in keys] + list(new)


def write_table(rows, path: str) -> None:
    with open(path, "w") as fh:
        fh.write("# libsalt tuning table, written by paper_1109_1264_amd.autotune\n")
        fh.write("# kind route dtype log2n unroll nontemporal blocks   # best ms, GB/s\n")
        for kind, route, dtype, l, u, nt, b, t, g in rows:
            fh.write("%s %d %d %d %d %d %d   # %.4f ms %.0f GB/s\n" % (kind, route, dtype, l, u, nt, b, t, g))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "salt_tuning.txt"))
    ap.add_argument("--trees", default="copy,scale,fig1,axpy,tree5,abc,t4,t5")
    ap.add_argument("--dtypes", default="f64,f32,bf16,f16")
    ap.add_argument("--log2n", default="10-28")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--step", type=int, default=1, help="tune every step-th log2 size")
    ap.add_argument("--kinds", default="eval,dot,nrm2,interp,jit,dotx,nrm2x,dotj,nrm2j,pairs,batch,batchj")
    ap.add_argument("--merge", action="store_true",
                    help="keep the rows of --out whose (kind, route, dtype) this run does not tune")
    ap.add_argument("--json", default=None, help="also write all rows as JSON here")
    ap.add_argument("--rotate", action="store_true",
                    help="time working sets of 4 MiB .. 1 GiB streaming from HBM (buffer slices cycled) "
                         "instead of cache-resident")
    ap.add_argument("--rotate-from-mib", type=int, default=4,
                    help="with --rotate, only working sets of at least this many MiB are streamed; smaller "
                         "ones are timed cache-resident")
    args = ap.parse_args(argv)
    lo, hi = (int(v) for v in args.log2n.split("-"))
    sizes = list(range(lo, hi + 1, args.step))
    if sizes[-1] != hi:
        sizes.append(hi)
    kinds = args.kinds.split(",")
    rf = args.rotate_from_mib << 20
    t0 = time.time()
    rows = []
    for dname in args.dtypes.split(","):
        d = DT_NAMES[dname]
        for kind in ("dot", "nrm2"):
            if kind in kinds:
                rows += tune(kind, None, d, sizes, args.reps, verbose=True, rotate=args.rotate, rotate_from=rf)
        if "eval" in kinds:
            for tree in args.trees.split(","):
                rows += tune("eval", tree, d, sizes, args.reps, verbose=True, rotate=args.rotate, rotate_from=rf)
        for kind in ("interp", "jit", "dotx", "nrm2x", "dotj", "nrm2j"):
            if kind in kinds:
                rows += tune(kind, None, d, sizes, args.reps, verbose=True, rotate=args.rotate, rotate_from=rf)
        if "pairs" in kinds:
            for i in range(len(PAIRS)):
                rows += tune("pair%d" % i, None, d, sizes, args.reps, verbose=True, rotate=args.rotate,
                             rotate_from=rf)
    if "batch" in kinds:
        from . import workloads

        c4 = [workloads.batch_lengths(4096, seed=workloads.SEED_BATCHED),
              workloads.batch_lengths(512, seed=workloads.SEED_BATCHED + 1)]
        rows += tune_batch("abc", S.F32, c4, with_dot=True, reps=args.reps, verbose=True)
        for dname in ("f32", "bf16", "f64"):
            for tree in ("fig1", "axpy", "tree5", "t4", "t5"):
                rows += tune_batch(tree, DT_NAMES[dname], serving_scenarios(), with_dot=False,
                                   reps=args.reps, verbose=True)
    if "batchj" in kinds:  # batched launches of compiled trees
        for dname in ("f32", "bf16", "f64"):
            rows += tune_batch("compiled", DT_NAMES[dname], serving_scenarios(), with_dot=False,
                               reps=args.reps, verbose=True)
    if args.merge and os.path.exists(args.out):
        rows = merged(read_table(args.out), rows)
    write_table(rows, args.out)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rows, fh)
    print("wrote %d rows to %s in %.0f s" % (len(rows), args.out, time.time() - t0), file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
