"""Benchmark of the SALT hot path on one MI355X.

One step = one pass of the hot path over one batch of HBM-resident synthetic
vectors (the BLAS-1 sweep at its largest size, n = 2^28, binary64):
    d = a*b + c*e - f      (fused 5-operand tree, salt_eval)
    d = alpha*a + d        (salt_axpy, in place)
    dot(a, b)              (salt_dot)
    nrm2(c)                (salt_nrm2)
`value` = algorithmic bytes of the step (inputs read once + outputs written
once: 96 B per element) / wall time per step, in GB/s. Per-kernel durations
are HIP events recorded on the launch stream around every launch inside the
timed region.

The same JSON line also reports the whole size sweep and the three systems
layers beside the plain binary64 kernels (each measured after the timed
step):
    mix:       each read/write mix (1..6 reads with one write; 1, 2, 3, 5
               reads alone) on 2^28 binary64 elements: a plain stream
               reference kernel beside the library kernel with that mix; the
               5-read 1-write reference is the roofline's mix ceiling;
    sweep:     axpy, dot, nrm2 and the 5-operand tree for n = 2^10 .. 2^28 in
               binary64 and binary32 (device time per launch, GB/s, % of
               8 TB/s, % of the copy tree's rate at the same n, and whether
               the working set is past the last-level cache), and the host
               time per small call of the binding and the expression front
               end (host_enqueue_us);
    fusion:    one fused pass against the same result composed from
               single-operation calls (out-of-place scale, a + (b - c),
               dot of two trees), with identical bits; and the Fig. 1 tree
               at n = 2^20 (cache-resident and with rotated buffers);
    precision: dot / nrm2 at n = 2^26, storage FP64 / FP32 / BF16, with the
               error against the binary64 oracle per result;
    blas1:     asum, iamax, scal and the strided routines at increments 2, 4;
    vendor:    rocBLAS axpy, dot, nrm2, copy, scal at n = 2^28 (binary64,
               binary32) beside the library's, on the same buffers and stream;
    batched:   4096 lognormal-length instances of alpha*a + (b - c) plus
               dot(a, b) in one persistent launch replayed from a HIP graph,
               against 4096 separate launches and one binary64 kernel;
    served:    Poisson request streams over five trees (binary32 / bfloat16 /
               binary64 mix, lengths 2^8..2^24, 64 GB resident pool) at
               fractions of the measured saturation rate: p50 / p99 latency
               and throughput; then one more stream served with kept outputs,
               each request's output checked bit for bit against the oracle
               on sampled elements (served_parity_ok).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--log2n 28]
                    [--sections main,mix,sweep,fusion,precision,blas1,vendor,batched,served]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "achieved HBM GB/s (% of peak) on fused vector exprs; served p50/p99 latency"
PROFILE_PMC = os.path.join(ROOT, "profiles", "pmc_tree5_f64_n2p28.json")


_T0 = time.perf_counter()


def log(*a):
    print("[%6.1f s]" % (time.perf_counter() - _T0), *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the tree kernel's sources (the template, its element types and
    tree nodes, and its launcher)."""
    h = hashlib.sha256()
    for f in ("eval_tree.hpp", "device.hpp", "expr.hpp", "eval.hip"):
        with open(os.path.join(ROOT, "paper_1109_1264_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(n_elems: int):
    """HBM bytes per launch of the tree kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source and with
    the library's current split of the call into dispatches."""
    if not os.path.exists(PROFILE_PMC):
        return None
    with open(PROFILE_PMC) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("n") != n_elems:
        return None
    import paper_1109_1264_amd.salt as salt

    if salt.salt_eval_chunking(5, n_elems, salt.F64)[1] != d.get("dispatches_per_launch"):
        return None
    return d.get("traffic_bytes_per_launch")


def event_ms(fn, reps: int, warm: int = 2) -> float:
    """Mean duration (ms) of fn() from HIP events on the current stream."""
    import numpy as np
    import torch

    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the step
# ---------------------------------------------------------------------------

def host_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the share of the host given to one
    GPU)."""
    try:
        t = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        t = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        t = min(t, int(env))
    return max(1, t)


def cpu_baseline(log2n_sample: int, reps: int = 5):
    """The oracle timed on the host: one step of the hot path (the 5-operand
    tree, axpy, and the plain binary64 dot and nrm2 loops) on a bounded sample
    of the GPU step's elements, with one thread and with every thread this
    process may use (OpenMP shares of the element range, inputs first touched
    by the same split). Dot2, the reference-value reduction, is timed apart."""
    import numpy as np

    import oracle
    from paper_1109_1264_amd import workloads

    n = 1 << log2n_sample
    a0, b0, c0, e0, f0 = workloads.uniform(n, "f64", workloads.sweep_seed(n), 5)
    alpha = workloads.alpha(workloads.sweep_seed(n))
    tree5 = [1, (1 << 8) | 1, 5, (2 << 8) | 1, (3 << 8) | 1, 5, 3, (4 << 8) | 1, 4]
    threads = host_threads()

    def run(T):
        ops = [oracle.first_touch_copy(v, T) for v in (a0, b0, c0, e0, f0)]
        a, b, c, e, f = ops
        oracle.set_threads(T)
        times, used = [], 1
        try:
            for _ in range(reps):
                t0 = time.perf_counter()
                d = oracle.eval_program(tree5, ops, [], "f64")
                d = oracle.axpy(alpha, a, d, "f64")
                _, used = oracle.naive_dot_par(a, b, T)
                math.sqrt(oracle.naive_dot_par(c, c, T)[0])
                times.append(time.perf_counter() - t0)
        finally:
            oracle.set_threads(1)
        return float(np.median(times)), used

    t1, _ = run(1)
    tn, used = run(threads) if threads > 1 else (t1, 1)
    t0 = time.perf_counter()
    oracle.dot2(a0, b0)
    oracle.nrm2(c0)
    t_dot2 = time.perf_counter() - t0
    gbps = lambda t: round(96.0 * n / t / 1e9, 3)
    return {"value": gbps(tn), "unit": "GB/s", "cores": used, "kind": "oracle",
            "sample": "one step of the same hot path (d = a*b + c*e - f, y = alpha*x + y, plain binary64 "
                      "dot and nrm2 loops) on n=2^%d binary64 elements (of the 2^28 in the GPU step), "
                      "median of %d runs, %d OpenMP threads (static shares, inputs first-touched by the "
                      "same split)" % (log2n_sample, reps, used),
            "seconds_per_step": round(tn, 4),
            "one_thread": {"value": gbps(t1), "seconds_per_step": round(t1, 4)},
            "dot2_reference_seconds": {"dot_and_nrm2": float("%.4g" % t_dot2), "threads": 1,
                                       "what": "Dot2 (compensated) dot(a, b) and nrm2(c), the reference "
                                               "values of the parity checks, timed apart"},
            "host": host_cpu()}


def host_cpu() -> dict:
    """The host's CPU model, sockets and logical CPU count (the baseline's
    machine)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    lscpu = {}
    try:
        import subprocess

        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                lscpu[k.strip()] = v.strip()
    except Exception:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "threads_allowed": host_threads(),
            "lscpu": lscpu}


# ---------------------------------------------------------------------------
# main step (BLAS-1 sweep, largest size)
# ---------------------------------------------------------------------------

def section_main(args, out):
    import numpy as np
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    dev = torch.device("cuda:0")
    n = 1 << args.log2n
    seed = workloads.sweep_seed(n)
    log("bench: generating 5 x %d binary64 operands on the device (seed %d)" % (n, seed))
    a, b, c, e, f = workloads.uniform_device(n, "f64", seed, 5, device=dev)
    alpha = workloads.alpha(seed)
    d = torch.empty(n, dtype=torch.float64, device=dev)
    ws = salt.workspace(n, salt.F64, dev)
    r_dot = torch.empty(1, dtype=torch.float64, device=dev)
    r_nrm = torch.empty(1, dtype=torch.float64, device=dev)
    T = salt.token
    tree5 = [T(salt.LOAD, 0), T(salt.LOAD, 1), T(salt.MUL), T(salt.LOAD, 2), T(salt.LOAD, 3), T(salt.MUL),
             T(salt.ADD), T(salt.LOAD, 4), T(salt.SUB)]
    copy = [T(salt.LOAD, 0)]
    bytes_per_elem = {"tree5": 48, "axpy": 24, "dot": 16, "nrm2": 8}
    names = list(bytes_per_elem)

    def launch(k):
        if k == "tree5":
            salt.salt_eval(tree5, [a, b, c, e, f], [], d)
        elif k == "axpy":
            salt.salt_axpy(alpha, a, d)
        elif k == "dot":
            salt.salt_dot(a, b, result=r_dot, ws=ws)
        elif k == "nrm2":
            salt.salt_nrm2(c, result=r_nrm, ws=ws)
        else:
            salt.salt_eval(copy, [a], [], d)

    if args.kernels_only:
        for k in args.kernels_only.split(","):
            for _ in range(args.steps):
                launch(k)
            torch.cuda.synchronize()
            log("bench: ran %s x%d" % (k, args.steps))
        return None

    def step(events=None):
        for k in names:
            if events is not None:
                events[k][0].record()
            launch(k)
            if events is not None:
                events[k][1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in names}
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = {k: float(np.mean([ev[s][k][0].elapsed_time(ev[s][k][1]) for s in range(args.steps)])) for k in names}
    step_bytes = sum(bytes_per_elem.values()) * n
    value = step_bytes / (wall / args.steps) / 1e9

    copy_ms = event_ms(lambda: launch("copy"), 20)
    copy_gbps = 16.0 * n / (copy_ms * 1e-3) / 1e9
    # references outside this library, on the same buffers: torch's own copy
    # (the framework's bandwidth ceiling for one read + one write stream) and
    # the tree as five unfused torch operations (each intermediate goes
    # through HBM)
    torch_copy_ms = event_ms(lambda: d.copy_(a), 20)
    torch_tree_ms = event_ms(lambda: torch.sub(torch.add(torch.mul(a, b), torch.mul(c, e)), f, out=d), 10)
    # a call of the 5-operand tree runs as chunked launches (salt_eval_chunking),
    # each with the knobs of its own size
    chunking = {k: salt.salt_eval_chunking({"tree5": 5, "axpy": 2}[k], n, salt.F64) if k in ("tree5", "axpy")
                else (n, 1) for k in names}
    kernels = {k: {"avg_ms": round(per[k], 4), "GBps": round(bytes_per_elem[k] * n / (per[k] * 1e-3) / 1e9, 1),
                   "bytes_per_elem": bytes_per_elem[k],
                   "launches_per_call": chunking[k][1], "elems_per_launch": chunking[k][0],
                   "launch_config": salt.salt_tuning_lookup(0 if k in ("tree5", "axpy") else (1 if k == "dot" else 2),
                                                            {"tree5": 4, "axpy": 3}.get(k, -1), salt.F64,
                                                            chunking[k][0])}
               for k in names}
    achieved = bytes_per_elem["tree5"] * n / (per["tree5"] * 1e-3) / 1e9
    out.update({
        "value": round(value, 1), "ms_per_step": round(1e3 * wall / args.steps, 4),
        "config": {"workload": "BLAS-1 sweep, largest size: d=a*b+c*e-f, y=alpha*x+y, dot(x,y), nrm2(x); "
                               "binary64, n=2^%d, uniform[-1,1) operands resident in HBM" % args.log2n,
                   "n": n, "seed": seed, "alpha": alpha, "step_bytes": step_bytes},
        "pct_of_hbm_peak": round(100.0 * value / HBM_PEAK_GBPS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic_from_profile(n),
                     "kernel": "k_eval_tree<tree5, f64> (d = a*b + c*e - f)",
                     "launch": "one salt_eval call over n elements: %d dispatches of %d elements in sequence "
                               "on one stream, timed together" % (chunking["tree5"][1], chunking["tree5"][0]),
                     "algorithmic_bytes_per_launch": bytes_per_elem["tree5"] * n},
        "kernels": kernels,
        "copy_ceiling": {"avg_ms": round(copy_ms, 4), "GBps": round(copy_gbps, 1),
                         "pct_of_hbm_peak": round(100 * copy_gbps / HBM_PEAK_GBPS, 2)},
        "torch_reference": {"copy_ms": round(torch_copy_ms, 4),
                            "copy_GBps": round(16.0 * n / (torch_copy_ms * 1e-3) / 1e9, 1),
                            "tree5_unfused_ms": round(torch_tree_ms, 4),
                            "tree5_fused_speedup": round(torch_tree_ms / per["tree5"], 3)},
    })
    if not args.no_parity:
        out["parity"] = main_parity(n, a, b, c, e, f, d, r_dot, r_nrm, ws, tree5)
    del a, b, c, e, f, d
    torch.cuda.empty_cache()
    return out


def main_parity(n, a, b, c, e, f, d, r_dot, r_nrm, ws, tree5):
    """Sampled bit-exact check of the tree kernel, and full-length checks of
    dot / nrm2 against the oracle (tolerance of Dot2, and bit for bit against
    the replay of the summation order), at the benchmarked size."""
    import numpy as np
    import torch

    import oracle
    import paper_1109_1264_amd.salt as salt

    log("bench: parity at full size")
    salt.salt_eval(tree5, [a, b, c, e, f], [], d)
    salt.salt_dot(a, b, result=r_dot, ws=ws)
    salt.salt_nrm2(c, result=r_nrm, ws=ws)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(99))
    idx = np.unique(np.concatenate([rng.integers(0, n, 1 << 16), np.arange(1024), np.arange(n - 1024, n)]))
    ti = torch.from_numpy(idx).to(a.device)
    ops = [t.index_select(0, ti).cpu().numpy() for t in (a, b, c, e, f)]
    got = d.index_select(0, ti).cpu().numpy()
    want = oracle.eval_program(tree5, ops, [], "f64")
    eval_ok = bool(np.array_equal(got.view(np.uint64), want.view(np.uint64)))
    ah, bh, ch = a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    ref, abs_sum = oracle.dot2(ah, bh)
    dot_err = abs(float(r_dot.item()) - ref) / abs_sum
    nref = oracle.nrm2(ch)
    nrm_err = abs(float(r_nrm.item()) - nref) / nref
    # bit for bit against the oracle's replay of the fixed summation order
    dot_bits = float(r_dot.item()) == float(oracle.reduce_canonical("dot", ah, bh, "f64"))
    nrm_bits = float(r_nrm.item()) == float(oracle.reduce_canonical("nrm2", ch, None, "f64"))
    return {"tree5_sampled_bit_exact": eval_ok, "samples": int(len(idx)),
            "dot_rel_err": dot_err, "nrm2_rel_err": nrm_err, "tol": 1e-13,
            "dot_bits_equal_order_replay": dot_bits, "nrm2_bits_equal_order_replay": nrm_bits,
            "ok": bool(eval_ok and dot_err <= 1e-13 and nrm_err <= 1e-13 and dot_bits and nrm_bits)}


# ---------------------------------------------------------------------------
# size sweep (BLAS-1 sweep, every size)
# ---------------------------------------------------------------------------

def graph_ms(fn, reps: int) -> float:
    """Per-launch time of fn() from a captured graph of `reps` launches,
    replayed between two events: device time of back-to-back launches, free
    of Python launch overhead."""
    import torch

    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    g.replay()
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) / reps
    del g
    return t


def section_sweep(args):
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    T = salt.token
    tree5 = [T(salt.LOAD, 0), T(salt.LOAD, 1), T(salt.MUL), T(salt.LOAD, 2), T(salt.LOAD, 3), T(salt.MUL),
             T(salt.ADD), T(salt.LOAD, 4), T(salt.SUB)]
    out = {"timing": "per-launch device time from a replayed graph of back-to-back launches",
           "regime": "sizes whose working set is >= 1 GiB are HBM-bound; smaller ones run from the "
                     "256 MiB last-level cache, L2 or are launch-bound"}
    hi = args.log2n
    for name in ("f64", "f32"):
        code = salt.F64 if name == "f64" else salt.F32
        es = 8 if name == "f64" else 4
        log("bench: sweep %s 2^10..2^%d" % (name, hi))
        a, b, c, e, f = workloads.uniform_device(1 << hi, name, workloads.sweep_seed(1 << hi), 5)
        d = torch.empty(1 << hi, dtype=a.dtype, device="cuda")
        ws = salt.workspace(1 << hi, code)
        r = torch.empty(1, dtype=torch.float64 if name == "f64" else torch.float32, device="cuda")
        copy = [T(salt.LOAD, 0)]
        rows = {"axpy": [], "dot": [], "nrm2": [], "tree5": [], "copy": []}
        for l in range(10, hi + 1):
            n = 1 << l
            al = workloads.alpha(workloads.sweep_seed(n))
            v = [t[:n] for t in (a, b, c, e, f)]
            dn = d[:n]
            fns = {"copy": (lambda: salt.salt_eval(copy, v[:1], [], dn), 2),
                   "axpy": (lambda: salt.salt_axpy(al, v[0], dn), 3),
                   "dot": (lambda: salt.salt_dot(v[0], v[1], result=r, ws=ws), 2),
                   "nrm2": (lambda: salt.salt_nrm2(v[2], result=r, ws=ws), 1),
                   "tree5": (lambda: salt.salt_eval(tree5, v, [], dn), 6)}
            reps = 50 if l <= 20 else (10 if l <= 24 else 4)
            copy_gbps = None
            for k, (fn, arrays) in fns.items():
                t = graph_ms(fn, reps)
                nbytes = arrays * es * n
                gbps = nbytes / (t * 1e-3) / 1e9
                if k == "copy":
                    copy_gbps = gbps
                # % of HBM peak is meaningful only once the working set is well
                # past the 256 MiB last-level cache (>= 1 GiB)
                rows[k].append([l, round(t, 5), round(gbps, 1), round(100 * gbps / 8000, 1),
                                round(100 * gbps / copy_gbps, 1), nbytes >= (1 << 30)])
        out[name] = {k: {"columns": ["log2n", "ms", "GBps", "pct_of_8TBps", "pct_of_copy_same_n", "hbm_regime"],
                         "rows": v} for k, v in rows.items()}
        del a, b, c, e, f, d, ws
        torch.cuda.empty_cache()
    out["host_enqueue_us"] = host_enqueue_us()
    return out


def host_enqueue_us(n: int = 1024, calls: int = 2000) -> dict:
    """Host time per call to put one small call on the stream (the Python
    binding, the library's checks and knob lookup, and the HIP launches),
    with a torch element-wise op beside it; n binary64 elements, so the
    device keeps up and the host is what is timed."""
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads
    from paper_1109_1264_amd.expr import Vec, expression

    T = salt.token
    tree5 = [T(salt.LOAD, 0), T(salt.LOAD, 1), T(salt.MUL), T(salt.LOAD, 2), T(salt.LOAD, 3), T(salt.MUL),
             T(salt.ADD), T(salt.LOAD, 4), T(salt.SUB)]
    v = workloads.uniform_device(n, "f64", 91, 5)
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    ws = salt.workspace(n, salt.F64)
    r = torch.empty(1, dtype=torch.float64, device="cuda")
    a, b, c, e, f = (Vec(t) for t in v)
    dv = Vec(d)
    t5 = expression(lambda a, b, c, e, f: a * b + c * e - f)
    fns = {"salt_eval tree5": lambda: salt.salt_eval(tree5, v, [], d),
           "operators d[:] = a*b + c*e - f (tree built per call)": lambda: dv.__setitem__(slice(None),
                                                                                         a * b + c * e - f),
           "expression(...) built once, called": lambda: t5(d, *v),
           "salt_axpy": lambda: salt.salt_axpy(1.5, v[0], d),
           "salt_dot (two kernels)": lambda: salt.salt_dot(v[0], v[1], result=r, ws=ws),
           "torch.add (reference)": lambda: torch.add(v[0], v[1], out=d)}
    res = {}
    for k, fn in fns.items():
        for _ in range(50):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(calls):
            fn()
        t1 = time.perf_counter()
        torch.cuda.synchronize()
        res[k] = round((t1 - t0) / calls * 1e6, 2)
    return {"n": n, "dtype": "f64", "calls": calls, "us_per_call": res}


# ---------------------------------------------------------------------------
# the vendor BLAS on the same GPU (context: the paper compares with BLAS)
# ---------------------------------------------------------------------------

def section_vendor(args):
    """rocBLAS level-1 routines (axpy, dot, nrm2, copy, scal) at n = 2^28 in
    binary64 and binary32, beside the library's own on the same buffers,
    both timed with HIP events on the same stream (the paper's comparison
    is against CPU BLAS, Sec. 5; this is the GPU's vendor BLAS). Results
    are not compared: rocBLAS's summation order is its own."""
    import ctypes

    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    try:
        rb = ctypes.CDLL("librocblas.so")
    except OSError as e:
        return {"available": False, "why": str(e)}
    h = ctypes.c_void_p()
    if rb.rocblas_create_handle(ctypes.byref(h)) != 0:
        return {"available": False, "why": "rocblas_create_handle failed"}
    n = 1 << args.log2n
    log("bench: rocBLAS level-1 beside the library, n = 2^%d" % args.log2n)
    P = ctypes.c_void_p
    out = {"available": True, "n": n,
           "columns": ["rocblas_ms", "rocblas_GBps", "library_ms", "library_GBps", "library_over_rocblas"]}
    cat = dict(salt.salt_catalogue())
    try:
        if rb.rocblas_set_stream(h, P(torch.cuda.current_stream().cuda_stream)) != 0:
            return {"available": False, "why": "rocblas_set_stream failed"}
        for dt, code, es, pre, cty in (("f64", salt.F64, 8, "d", ctypes.c_double),
                                       ("f32", salt.F32, 4, "s", ctypes.c_float)):
            x, y = workloads.uniform_device(n, dt, workloads.sweep_seed(n) + 9, 2)
            res = torch.empty(1, dtype=x.dtype, device="cuda")
            ws = salt.workspace(n, code)
            alpha = cty(1.25)
            f = {k: getattr(rb, "rocblas_%s%s" % (pre, k)) for k in ("axpy", "dot", "nrm2", "copy", "scal")}
            px, py, pr = P(x.data_ptr()), P(y.data_ptr()), P(res.data_ptr())

            def call(st):
                if st != 0:
                    raise RuntimeError("rocBLAS status %d" % st)

            vendor = {
                "axpy": lambda: (rb.rocblas_set_pointer_mode(h, 0),
                                 call(f["axpy"](h, ctypes.c_int(n), ctypes.byref(alpha), px, 1, py, 1))),
                "dot": lambda: (rb.rocblas_set_pointer_mode(h, 1), call(f["dot"](h, ctypes.c_int(n), px, 1, py, 1, pr))),
                "nrm2": lambda: (rb.rocblas_set_pointer_mode(h, 1), call(f["nrm2"](h, ctypes.c_int(n), px, 1, pr))),
                "copy": lambda: call(f["copy"](h, ctypes.c_int(n), px, 1, py, 1)),
                "scal": lambda: (rb.rocblas_set_pointer_mode(h, 0),
                                 call(f["scal"](h, ctypes.c_int(n), ctypes.byref(alpha), py, 1))),
            }
            ours = {"axpy": lambda: salt.salt_axpy(1.25, x, y),
                    "dot": lambda: salt.salt_dot(x, y, result=res, ws=ws),
                    "nrm2": lambda: salt.salt_nrm2(x, result=res, ws=ws),
                    "copy": lambda: salt.salt_eval(cat["copy"], [x], [], y),
                    "scal": lambda: salt.salt_scal(1.25, y, n)}
            nbytes = {"axpy": 3, "dot": 2, "nrm2": 1, "copy": 2, "scal": 2}
            rows = {}
            for k in ours:
                t_v = event_ms(vendor[k], 10)
                t_o = event_ms(ours[k], 10)
                b = nbytes[k] * es * n
                rows[k] = [round(t_v, 4), round(b / (t_v * 1e-3) / 1e9, 1), round(t_o, 4),
                           round(b / (t_o * 1e-3) / 1e9, 1), round(t_v / t_o, 3)]
            out[dt] = rows
            del x, y, ws
            torch.cuda.empty_cache()
    finally:
        rb.rocblas_destroy_handle(h)
    return out


# ---------------------------------------------------------------------------
# read/write mix: the plain stream reference beside the library's kernels
# ---------------------------------------------------------------------------

def section_mix(args):
    """Bandwidth of each read/write mix on binary64 arrays of 2^28 elements
    (2 GiB each, HBM-resident): the plain stream reference (one 16-byte
    chunk per lane, integer xor, no loop) against the library kernel with
    the same mix (catalogue trees reading k operands and writing one; dot,
    nrm2 and nrm2 of a sum of 3 or 5 operands on its run-time compiled
    kernel, reading only). The reference
    at 5 reads and 1 write is the ceiling the fused 5-operand tree is held
    to."""
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    n = 1 << args.log2n
    log("bench: read/write mix, n = 2^%d binary64" % args.log2n)
    ins = workloads.uniform_device(n, "f64", workloads.sweep_seed(n) + 3, 6)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ws = salt.workspace(n, salt.F64)
    r = torch.empty(1, dtype=torch.float64, device="cuda")
    cat = dict(salt.salt_catalogue())
    # the sums of operands are not catalogue pairs: their norms run on
    # kernels compiled at run time for them (compiled here, before timing)
    for k in (3, 5):
        salt.salt_jit_compile_reduce(sum_prog(k), None, k, 0, salt.F64)
    lib = {(1, 1): ("copy", lambda: salt.salt_eval(cat["copy"], ins[:1], [], out)),
           (2, 1): ("axpy tree", lambda: salt.salt_eval(cat["axpy"], ins[:2], [1.25], out)),
           (3, 1): ("fig1 tree", lambda: salt.salt_eval(cat["fig1"], ins[:3], [], out)),
           (4, 1): ("t4 tree", lambda: salt.salt_eval(cat["t4"], ins[:4], [1.25], out)),
           (5, 1): ("tree5", lambda: salt.salt_eval(cat["tree5"], ins[:5], [], out)),
           (6, 1): ("t5 tree", lambda: salt.salt_eval(cat["t5"], ins[:6], [1.25], out)),
           (1, 0): ("nrm2", lambda: salt.salt_nrm2(ins[0], result=r, ws=ws)),
           (2, 0): ("dot", lambda: salt.salt_dot(ins[0], ins[1], result=r, ws=ws)),
           (3, 0): ("nrm2(a+b+c), compiled",
                    lambda: salt.salt_nrm2_expr(sum_prog(3), ins[:3], [], result=r, ws=ws)),
           (5, 0): ("nrm2(a+b+c+e+f), compiled",
                    lambda: salt.salt_nrm2_expr(sum_prog(5), ins[:5], [], result=r, ws=ws))}
    rows = []
    for (R, W), (name, fn) in lib.items():
        nbytes = (R + W) * 8 * n
        t_ref = event_ms(lambda: salt.salt_stream_reference(ins[:R], out if W else None), 6)
        t_lib = event_ms(fn, 6)
        g_ref = nbytes / (t_ref * 1e-3) / 1e9
        g_lib = nbytes / (t_lib * 1e-3) / 1e9
        rows.append([R, W, round(t_ref, 4), round(g_ref, 1), round(100 * g_ref / HBM_PEAK_GBPS, 1), name,
                     round(t_lib, 4), round(g_lib, 1), round(g_lib / g_ref, 3)])
    del ins, out, ws
    torch.cuda.empty_cache()
    return {"n": n, "dtype": "f64",
            "reference": "salt_stream_reference: one 16-byte chunk per lane, integer xor of the inputs, "
                         "non-temporal loads and stores, no loop",
            "columns": ["reads", "writes", "ref_ms", "ref_GBps", "ref_pct_of_8TBps", "library_kernel",
                        "lib_ms", "lib_GBps", "lib_over_ref"],
            "rows": rows}


# ---------------------------------------------------------------------------
# fusion against composition of single-operation calls
# ---------------------------------------------------------------------------

def section_fusion(args):
    """The paper's out-of-place scale experiment (Sec. 5, Fig. 6: BLAS needs a
    copy and a scal) and two more trees, fused into one pass against the same
    results composed from single-operation kernels; results are checked for
    identical bits."""
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    n = 1 << args.log2n
    log("bench: fusion vs composition, n = 2^%d" % args.log2n)
    T = salt.token
    L0, L1, L2 = T(salt.LOAD, 0), T(salt.LOAD, 1), T(salt.LOAD, 2)
    a, b, c, e = workloads.uniform_device(n, "f64", workloads.sweep_seed(n) + 1, 4)
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    t = torch.empty(n, dtype=torch.float64, device="cuda")
    ws = salt.workspace(n, salt.F64)
    r1 = torch.empty(1, dtype=torch.float64, device="cuda")
    r2 = torch.empty(1, dtype=torch.float64, device="cuda")
    al = workloads.alpha(7)
    scale = [T(salt.SCALAR, 0), L0, T(salt.MUL)]
    cases = {
        "scale_out_of_place": {
            "fused": (lambda: salt.salt_eval(scale, [a], [al], d), 16),
            "composed": (lambda: (salt.salt_eval([L0], [a], [], t), salt.salt_eval(scale, [t], [al], t)), 32),
            "what": "d = alpha*a: one pass vs copy then in-place scale"},
        "fig1": {
            "fused": (lambda: salt.salt_eval([L0, L1, L2, T(salt.SUB), T(salt.ADD)], [a, b, c], [], d), 32),
            "composed": (lambda: (salt.salt_eval([L0, L1, T(salt.SUB)], [b, c], [], t),
                                  salt.salt_eval([L0, L1, T(salt.ADD)], [a, t], [], t)), 48),
            "what": "d = a + (b - c): one pass vs t = b - c, d = a + t"},
        "dot_of_trees": {
            "fused": (lambda: salt.salt_dot_expr([L0, L1, T(salt.ADD)], [L0, L1, T(salt.SUB)], [c, e], [],
                                                 result=r1, ws=ws), 16),
            "composed": (lambda: (salt.salt_eval([L0, L1, T(salt.ADD)], [c, e], [], d),
                                  salt.salt_eval([L0, L1, T(salt.SUB)], [c, e], [], t),
                                  salt.salt_dot(d, t, result=r2, ws=ws)), 48),
            "what": "dot(c + e, c - e): one pass vs two evaluations and a dot"},
    }
    out = {"n": n, "dtype": "f64"}
    for name, cs in cases.items():
        tf = event_ms(cs["fused"][0], 10)
        fused_bits = (d.clone() if name != "dot_of_trees" else r1.clone())
        tc = event_ms(cs["composed"][0], 10)
        comp_bits = (t if name != "dot_of_trees" else r2)
        torch.cuda.synchronize()
        same = bool(torch.equal(fused_bits.view(torch.int64), comp_bits.view(torch.int64)))
        out[name] = {"what": cs["what"], "fused_ms": round(tf, 4), "composed_ms": round(tc, 4),
                     "speedup": round(tc / tf, 3), "fused_bytes_per_elem": cs["fused"][1],
                     "composed_bytes_per_elem": cs["composed"][1],
                     "fused_GBps": round(cs["fused"][1] * n / (tf * 1e-3) / 1e9, 1),
                     "composed_GBps": round(cs["composed"][1] * n / (tc * 1e-3) / 1e9, 1),
                     "same_bits": same}
    del a, b, c, e, d, t, ws
    torch.cuda.empty_cache()
    out["fig1_n2p20"] = fig1_small()
    out["expression_reductions"] = expression_reductions(args)
    out["compiled_trees"] = compiled_trees()
    return out


def compiled_trees():
    """A tree outside the catalogue, (a + b) * c, on the interpreter against
    its run-time compiled kernel, by element type and size (device time per
    launch of back-to-back launches, buffers reused), with identical bits."""
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    T = salt.token
    prog = [T(salt.LOAD, 0), T(salt.LOAD, 1), T(salt.ADD), T(salt.LOAD, 2), T(salt.MUL)]
    out = {"tree": "(a + b) * c", "bytes": "4 s bytes per element (3 reads, 1 write)"}
    log("bench: compiled trees")
    t0 = time.perf_counter()
    for dt in ("f64", "f32", "bf16"):
        salt.salt_jit_compile(prog, 3, 0, {"f64": salt.F64, "f32": salt.F32, "bf16": salt.BF16}[dt])
    out["compile_seconds_three_types"] = round(time.perf_counter() - t0, 3)
    for dt in ("f64", "f32", "bf16"):
        es = {"f64": 8, "f32": 4, "bf16": 2}[dt]
        rows = []
        for l in (20, 22, 24, 26, 28):
            n = 1 << l
            a, b, c = workloads.uniform_device(n, dt, workloads.sweep_seed(n) + 5, 3)
            d1 = torch.empty(n, dtype=a.dtype, device="cuda")
            d2 = torch.empty(n, dtype=a.dtype, device="cuda")
            reps = 20 if l <= 24 else 4
            salt.salt_jit_set_mode(salt.JIT_OFF)
            t_int = graph_ms(lambda: salt.salt_eval(prog, [a, b, c], [], d1), reps)
            salt.salt_jit_set_mode(salt.JIT_EXPLICIT)
            t_jit = graph_ms(lambda: salt.salt_eval(prog, [a, b, c], [], d2), reps)
            salt.salt_jit_set_mode(salt.JIT_AUTO)
            torch.cuda.synchronize()
            same = bool(torch.equal(d1.view(torch.uint8), d2.view(torch.uint8)))
            gb = lambda t: round(4 * es * n / (t * 1e-3) / 1e9, 1)
            rows.append([l, round(t_int, 5), gb(t_int), round(t_jit, 5), gb(t_jit), same])
            del a, b, c, d1, d2
            torch.cuda.empty_cache()
        out[dt] = {"columns": ["log2n", "interpreter_ms", "interpreter_GBps", "compiled_ms", "compiled_GBps",
                               "same_bits"], "rows": rows}
    return out


def expression_reductions(args):
    """Trees reduced without being written (Sec. 2's lazy evaluation inside
    a dot product or a norm), n = 2^28, by storage type: the pairs with
    ahead-of-time kernels against an equivalent pair (b + a for a + b: the
    same bits) on the interpreter and on its run-time compiled kernel, and
    the same bits checked."""
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    T = salt.token
    L0, L1, S0 = T(salt.LOAD, 0), T(salt.LOAD, 1), T(salt.SCALAR, 0)
    n = 1 << args.log2n
    cases = {"dot(a+b, a-b)": (([L0, L1, T(salt.ADD)], [L0, L1, T(salt.SUB)]),
                               ([L1, L0, T(salt.ADD)], [L0, L1, T(salt.SUB)])),
             "nrm2(alpha*a + b)": (([S0, L0, T(salt.MUL), L1, T(salt.ADD)], None),
                                   ([L1, S0, L0, T(salt.MUL), T(salt.ADD)], None))}
    out = {"n": n, "bytes": "2 operands read once: 2 s bytes per element"}
    for dt in ("f64", "f32", "bf16"):
        code = {"f64": salt.F64, "f32": salt.F32, "bf16": salt.BF16}[dt]
        es = {"f64": 8, "f32": 4, "bf16": 2}[dt]
        log("bench: expression reductions, %s" % dt)
        a, b = workloads.uniform_device(n, dt, workloads.sweep_seed(n) + 4, 2)
        ws = salt.workspace(n, code)
        rdt = torch.float64 if dt == "f64" else torch.float32
        r1 = torch.empty(1, dtype=rdt, device="cuda")
        r2 = torch.empty(1, dtype=rdt, device="cuda")
        r3 = torch.empty(1, dtype=rdt, device="cuda")
        rows = {}
        for name, ((px, py), (qx, qy)) in cases.items():
            def run(p, q, r):
                if q is None:
                    salt.salt_nrm2_expr(p, [a, b], [1.375], result=r, ws=ws)
                else:
                    salt.salt_dot_expr(p, q, [a, b], [1.375], result=r, ws=ws)
            t_aot = event_ms(lambda: run(px, py, r1), 10)
            try:
                salt.salt_jit_set_mode(salt.JIT_OFF)
                t_int = event_ms(lambda: run(qx, qy, r2), 10)
                salt.salt_jit_set_mode(salt.JIT_EXPLICIT)
                salt.salt_jit_compile_reduce(qx, qy, 2, 1, code)
                assert salt.salt_reduce_expr_route(qx, qy, 2, 1, code) == salt.ROUTE_COMPILED
                t_jit = event_ms(lambda: run(qx, qy, r3), 10)
            finally:
                salt.salt_jit_set_mode(salt.JIT_AUTO)
            torch.cuda.synchronize()
            gb = lambda t: round(2 * es * n / (t * 1e-3) / 1e9, 1)
            rows[name] = {"ahead_of_time_ms": round(t_aot, 4), "ahead_of_time_GBps": gb(t_aot),
                          "ahead_of_time_pct_of_8TBps": round(100 * 2 * es * n / (t_aot * 1e-3) / 8e12, 1),
                          "interpreter_ms": round(t_int, 4), "interpreter_GBps": gb(t_int),
                          "compiled_ms": round(t_jit, 4), "compiled_GBps": gb(t_jit),
                          "same_bits": bool(torch.equal(r1, r2) and torch.equal(r1, r3))}
        out[dt] = rows
        del a, b, ws
        torch.cuda.empty_cache()
    return out


def fig1_small() -> dict:
    """The Fig. 1 tree d = a + (b - c) at its own size (binary64, n = 2^20,
    32 MiB moved per launch): with the same buffers every launch (they stay
    in the 256 MiB last-level cache) and with 16 buffer sets cycled (512 MiB,
    so each launch streams from HBM)."""
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    T = salt.token
    fig1 = [T(salt.LOAD, 0), T(salt.LOAD, 1), T(salt.LOAD, 2), T(salt.SUB), T(salt.ADD)]
    n, sets = 1 << 20, 16
    bufs = [workloads.uniform_device(n, "f64", workloads.SEED_FIG1 + k, 3) for k in range(sets)]
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(sets)]
    t_res = graph_ms(lambda: salt.salt_eval(fig1, bufs[0], [], outs[0]), 64)
    state = {"k": 0}

    def rotated():
        k = state["k"] % sets
        state["k"] += 1
        salt.salt_eval(fig1, bufs[k], [], outs[k])
    t_rot = graph_ms(rotated, 64)
    nbytes = 32 * n
    del bufs, outs
    torch.cuda.empty_cache()
    return {"n": n, "dtype": "f64", "bytes_per_launch": nbytes,
            "resident_ms": round(t_res, 5), "resident_GBps": round(nbytes / (t_res * 1e-3) / 1e9, 1),
            "rotated_ms": round(t_rot, 5), "rotated_GBps": round(nbytes / (t_rot * 1e-3) / 1e9, 1),
            "rotated_pct_of_8TBps": round(100 * nbytes / (t_rot * 1e-3) / 8e12, 1),
            "rotation": "%d buffer sets (%d MiB) cycled launch by launch, beyond the last-level cache"
                        % (sets, sets * nbytes >> 20)}


# ---------------------------------------------------------------------------
# precision layer
# ---------------------------------------------------------------------------

def rotated_graph_ms(fns, reps: int) -> float:
    """Per-launch device time of a captured graph of `reps` launches that
    cycles through `fns` (one per buffer set): each launch reads a set that
    the launches in between have pushed out of the last-level cache."""
    state = {"k": 0}

    def step():
        fns[state["k"] % len(fns)]()
        state["k"] += 1
    return graph_ms(step, reps)


def section_precision(args):
    """dot and nrm2 at n = 2^26 with the operands stored in binary64, binary32
    and bfloat16 (ill-conditioned values), each from HBM: the timed launches
    cycle through copies of the operands (at least 4 sets and 2 GiB, so a
    set was evicted from the 256 MiB last-level cache before it is read
    again). Pass 1 alone (salt_reduce_partials) is timed beside the whole
    call, so the pass-2 launch is reported apart; the same call on one set
    (cache-resident where the set fits the cache) is reported as well."""
    import numpy as np
    import torch

    import oracle
    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    n = 1 << 26
    log("bench: precision layer, n = 2^26")
    x64, y64 = workloads.ill_conditioned(n, workloads.SEED_PRECISION)
    exact_dot, abs_dot = oracle.dot2(x64, y64)
    exact_nrm = oracle.nrm2(x64)
    rows = {}
    for name in ("f64", "f32", "bf16"):
        code = {"f64": salt.F64, "f32": salt.F32, "bf16": salt.BF16}[name]
        es = {"f64": 8, "f32": 4, "bf16": 2}[name]
        xs, ys = workloads.store(x64, name), workloads.store(y64, name)
        if name == "bf16":
            hx = torch.from_numpy(xs.view(np.int16)).view(torch.bfloat16)
            hy = torch.from_numpy(ys.view(np.int16)).view(torch.bfloat16)
        else:
            hx, hy = torch.from_numpy(xs), torch.from_numpy(ys)
        set_bytes = 2 * es * n
        sets = max(4, -(-(2 << 30) // set_bytes))
        dx = [hx.cuda() for _ in range(sets)]
        dy = [hy.cuda() for _ in range(sets)]
        ws = salt.workspace(n, code)
        tiles = salt.salt_reduce_workspace_bytes(n, code) // 8
        part = torch.empty(tiles, dtype=torch.float64, device="cuda")
        rdt = torch.float64 if name == "f64" else torch.float32
        r_dot = torch.empty(sets, dtype=rdt, device="cuda")
        r_nrm = torch.empty(sets, dtype=rdt, device="cuda")
        dots = [lambda k=k: salt.salt_dot(dx[k], dy[k], result=r_dot[k:k + 1], ws=ws) for k in range(sets)]
        nrms = [lambda k=k: salt.salt_nrm2(dx[k], result=r_nrm[k:k + 1], ws=ws) for k in range(sets)]
        p1_dot = [lambda k=k: salt.salt_reduce_partials(salt.MODE_DOT, dx[k], dy[k], partials=part)
                  for k in range(sets)]
        p1_nrm = [lambda k=k: salt.salt_reduce_partials(salt.MODE_NRM2, dx[k], partials=part) for k in range(sets)]
        reps = 8 * sets
        t_dot = rotated_graph_ms(dots, reps)
        t_nrm = rotated_graph_ms(nrms, reps)
        t_dot1 = rotated_graph_ms(p1_dot, reps)
        t_nrm1 = rotated_graph_ms(p1_nrm, reps)
        t_dot_res = graph_ms(dots[0], reps)
        t_nrm_res = graph_ms(nrms[0], reps)
        torch.cuda.synchronize()
        # every set holds the same values, so every set's result has the same bits
        same = bool(torch.equal(r_dot, r_dot[:1].expand(sets)) and torch.equal(r_nrm, r_nrm[:1].expand(sets)))
        got_dot, got_nrm = float(r_dot[0].item()), float(r_nrm[0].item())
        wx, wy = oracle.widen(xs, name), oracle.widen(ys, name)
        q_dot, q_abs = oracle.dot2(wx, wy)
        q_nrm = oracle.nrm2(wx)
        gb = lambda nbytes, t: round(nbytes / (t * 1e-3) / 1e9, 1)
        rows[name] = {
            "regime": "hbm: %d buffer sets (%d MiB) cycled launch by launch" % (sets, sets * set_bytes >> 20),
            "dot_ms": round(t_dot, 4), "dot_GBps": gb(2 * es * n, t_dot),
            "dot_pass1_ms": round(t_dot1, 4), "dot_pass1_GBps": gb(2 * es * n, t_dot1),
            "nrm2_ms": round(t_nrm, 4), "nrm2_GBps": gb(es * n, t_nrm),
            "nrm2_pass1_ms": round(t_nrm1, 4), "nrm2_pass1_GBps": gb(es * n, t_nrm1),
            "pass2_ms_approx": round(0.5 * ((t_dot - t_dot1) + (t_nrm - t_nrm1)), 4),
            "one_set_reused": {"what": "the same buffers every launch (set of %d MiB; %s)"
                                       % (set_bytes >> 20, "fits the 256 MiB last-level cache"
                                          if set_bytes <= (256 << 20) else "larger than the last-level cache"),
                               "dot_ms": round(t_dot_res, 4), "dot_GBps": gb(2 * es * n, t_dot_res),
                               "nrm2_ms": round(t_nrm_res, 4), "nrm2_GBps": gb(es * n, t_nrm_res)},
            "accumulation": "binary64 fma" if name == "f64" else
                            ("compensated binary32 (TwoProduct+TwoSum)" if name == "f32" else
                             "compensated binary32 (exact products, TwoSum)") + ", binary64 combine",
            # (i) end to end, including storage rounding, vs the binary64 data
            "dot_err_vs_f64_data": abs(got_dot - exact_dot) / abs_dot,
            "nrm2_err_vs_f64_data": abs(got_nrm - exact_nrm) / exact_nrm,
            # (ii) accumulation only, vs Dot2 on the stored values (the tolerance check)
            "dot_err_vs_stored": abs(got_dot - q_dot) / q_abs,
            "nrm2_err_vs_stored": abs(got_nrm - q_nrm) / q_nrm,
            "tol": oracle.TOL[name],
            "same_bits_every_set": same,
        }
        rows[name]["within_tol"] = bool(rows[name]["dot_err_vs_stored"] <= oracle.TOL[name]
                                        and rows[name]["nrm2_err_vs_stored"] <= oracle.TOL[name] and same)
        del dx, dy, ws, part
        torch.cuda.empty_cache()
    return {"n": n, "inputs": "random sign, log10|x| ~ U[-4,4] (seed 3000), stored with RNE",
            "timing": "per-launch device time from a replayed graph of back-to-back launches",
            "errors_are": "relative to sum|x_i y_i| (dot) or to the norm (nrm2)", "by_storage": rows}


# ---------------------------------------------------------------------------
# BLAS level-1 interface: asum, iamax and increments
# ---------------------------------------------------------------------------

def section_blas1(args):
    """asum and iamax (contiguous, HBM read-bound) and the strided routines at
    increments 2 and 4. Bytes are the algorithmic ones (elements the call
    reads and writes); a strided call moves whole 64- or 128-byte lines, so
    its useful bandwidth falls as the increment grows."""
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    n = 1 << args.log2n
    log("bench: BLAS level-1, n = 2^%d" % args.log2n)
    out = {"n": n, "dtype": "f64", "bytes": "algorithmic: 8 B per element read or written"}
    x, y = workloads.uniform_device(n, "f64", workloads.sweep_seed(n) + 2, 2)
    ws = salt.workspace(n, salt.F64)
    r = torch.empty(1, dtype=torch.float64, device="cuda")
    ri = torch.empty(1, dtype=torch.int64, device="cuda")
    rows = {
        "asum": (lambda: salt.salt_asum(x, n, 1, result=r, ws=ws), 8 * n),
        "iamax": (lambda: salt.salt_iamax(x, n, 1, result=ri, ws=ws), 8 * n),
        "nrm2": (lambda: salt.salt_nrm2(x, result=r, ws=ws), 8 * n),
        "scal": (lambda: salt.salt_scal(1.0, y, n, 1), 16 * n),
    }
    for inc in (2, 4):
        m = n // inc
        rows["dot_inc%d" % inc] = (lambda m=m, inc=inc: salt.salt_dot_strided(x, y, m, inc, inc, result=r, ws=ws),
                                   16 * m)
        rows["asum_inc%d" % inc] = (lambda m=m, inc=inc: salt.salt_asum(x, m, inc, result=r, ws=ws), 8 * m)
        rows["iamax_inc%d" % inc] = (lambda m=m, inc=inc: salt.salt_iamax(x, m, inc, result=ri, ws=ws), 8 * m)
        rows["axpy_inc%d" % inc] = (lambda m=m, inc=inc: salt.salt_axpy_strided(1.0, x, y, m, inc, inc), 24 * m)
        rows["copy_inc%d" % inc] = (lambda m=m, inc=inc: salt.salt_copy(x, y, m, inc, inc), 16 * m)
    for name, (fn, nbytes) in rows.items():
        t = event_ms(fn, 10)
        out[name] = {"ms": round(t, 4), "GBps": round(nbytes / (t * 1e-3) / 1e9, 1),
                     "frac_of_8TBps": round(nbytes / (t * 1e-3) / 8e12, 3)}
    del x, y, ws
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# batched layer
# ---------------------------------------------------------------------------

def section_batched(args):
    import numpy as np
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads
    from paper_1109_1264_amd.batch import Batch

    lengths = workloads.batch_lengths(4096, seed=workloads.SEED_BATCHED)
    total = int(lengths.sum())
    log("bench: batched layer, 4096 instances, %d elements" % total)
    offs = np.zeros(len(lengths) + 1, dtype=np.int64)
    offs[1:] = np.cumsum((lengths + 63) // 64 * 64)
    cap = int(offs[-1])
    a, b, c = workloads.uniform_device(cap, "f32", workloads.SEED_BATCHED, 3)
    d = torch.empty(cap, dtype=torch.float32, device="cuda")
    dots = torch.empty(len(lengths), dtype=torch.float32, device="cuda")
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_BATCHED + 1))
    alphas = rng.uniform(0.5, 2.0, len(lengths))
    T = salt.token
    abc = [T(salt.SCALAR, 0), T(salt.LOAD, 0), T(salt.MUL), T(salt.LOAD, 1), T(salt.LOAD, 2), T(salt.SUB),
           T(salt.ADD)]
    items = []
    for k, n in enumerate(lengths):
        s, e = int(offs[k]), int(offs[k]) + int(n)
        items.append({"n": int(n), "operands": [a[s:e], b[s:e], c[s:e]], "scalars": [float(alphas[k])],
                      "out": d[s:e], "dot_out": dots[k:k + 1]})
    bt = Batch(abc, items, salt.F32)
    g = bt.graph()
    alg_bytes = 16 * total + 8 * bt.tiles
    t_graph = event_ms(g.launch, 20)
    # the same two kernels launched directly (no graph), and 20 graph
    # launches back to back between one pair of events (the device time per
    # launch once the queue is ahead: no event-to-start latency)
    t_direct = event_ms(bt.launch, 20)
    g.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        g.launch()
    e1.record()
    torch.cuda.synchronize()
    t_b2b = e0.elapsed_time(e1) / 20
    # the same work as 4096 separate eval + dot calls
    ws = salt.workspace(1 << 20, salt.F32)

    def separate():
        for k, it in enumerate(items):
            salt.salt_eval(abc, it["operands"], it["scalars"], it["out"])
            salt.salt_dot(it["operands"][0], it["operands"][1], result=it["dot_out"], ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    separate()
    torch.cuda.synchronize()
    t_sep = 1e3 * (time.perf_counter() - t0)
    # one plain binary64 kernel over the same number of elements
    a64, b64, c64 = workloads.uniform_device(total, "f64", workloads.SEED_BATCHED, 3)
    d64 = torch.empty(total, dtype=torch.float64, device="cuda")
    r64 = torch.empty(1, dtype=torch.float64, device="cuda")
    ws64 = salt.workspace(total, salt.F64)

    def plain64():
        salt.salt_eval(abc, [a64, b64, c64], [1.25], d64)
        salt.salt_dot(a64, b64, result=r64, ws=ws64)
    t_64 = event_ms(plain64, 10)
    # where the time goes: the same workload split into its whole tiles and
    # its ragged last tiles (each as its own batch of items), and without
    # the fused dot
    tile_el = salt.salt_reduce_tile_elems(salt.F32)

    def sub_batch(lens, with_dot):
        its = []
        for k, n in enumerate(lens):
            if n <= 0:
                continue
            s0 = int(offs[k])
            its.append({"n": int(n), "operands": [a[s0:s0 + n], b[s0:s0 + n], c[s0:s0 + n]],
                        "scalars": [float(alphas[k])], "out": d[s0:s0 + n],
                        "dot_out": dots[k:k + 1] if with_dot else None})
        sb = Batch(abc, its, salt.F32)
        sg = sb.graph()
        t = event_ms(sg.launch, 20)
        el = int(sum(int(n) for n in lens if n > 0))
        r = {"items": len(its), "elements": el, "tiles": sb.tiles, "graph_ms": round(t, 4),
             "graph_GBps": round((16 * el + (8 * sb.tiles if with_dot else 0)) / (t * 1e-3) / 1e9, 1)}
        sg.close()
        sb.close()
        return r
    whole_lens = [(int(n) // tile_el) * tile_el for n in lengths]
    ragged_lens = [int(n) % tile_el for n in lengths]
    split = {"tile_elems": tile_el,
             "whole_tiles_only": sub_batch(whole_lens, True),
             "ragged_tiles_only": sub_batch(ragged_lens, True),
             "all_tiles_no_dot": sub_batch([int(n) for n in lengths], False)}
    res = {"instances": len(lengths), "elements": total, "tiles": bt.tiles, "split": split,
           "length_stats": {"min": int(lengths.min()), "median": int(np.median(lengths)),
                            "max": int(lengths.max()), "sigma_ln": 1.5},
           "graph_ms": round(t_graph, 4), "graph_GBps": round(alg_bytes / (t_graph * 1e-3) / 1e9, 1),
           "direct_launch_ms": round(t_direct, 4),
           "graph_back_to_back_ms": round(t_b2b, 4),
           "graph_back_to_back_GBps": round(alg_bytes / (t_b2b * 1e-3) / 1e9, 1),
           "launch_config": salt.salt_tuning_lookup(3, 5, salt.F32, total),
           "separate_launches_ms": round(t_sep, 3), "speedup_vs_separate": round(t_sep / t_graph, 1),
           "plain_f64_one_kernel_ms": round(t_64, 4),
           "plain_f64_GBps": round((32 * total + 16 * total) / (t_64 * 1e-3) / 1e9, 1)}
    g.close()
    bt.close()
    return res


# ---------------------------------------------------------------------------
# serving layer
# ---------------------------------------------------------------------------

def section_served(args):
    import torch

    from paper_1109_1264_amd import serve as V
    from paper_1109_1264_amd import workloads

    log("bench: served layer, building the resident pool")
    pool = V.Pool(args.pool_gb << 30, seed=workloads.SEED_SERVED)
    # 32 GB for outputs in flight: with 8 GB the arena, not the device, bounds
    # the saturated rate (about 4-5 TB/s instead of 5.5)
    arena_gb = 32
    arena, table = V.default_buffers(arena_bytes=arena_gb << 30, table_bytes=64 << 20)
    out = {"pool_GB": args.pool_gb, "arena_GB": arena_gb, "trees": list(V.TREES),
           "dtype_mix": dict(V.MIX), "lengths": "log-uniform 2^8..2^24"}
    # warm-up: the first calls load every batched kernel variant they meet
    # and touch the whole output arena
    trace, meta = V.make_trace(pool, 2000, seed=workloads.SEED_SERVED + 999, rate=None)
    for pol in (V.GROUP_MIXED, V.GROUP_BY_TREE):
        V.serve(trace, arena, table, grouping=pol)
    # saturation: every request present at t = 0; each grouping policy twice,
    # interleaved, the better run of each kept
    sat_trace, sat_meta = V.make_trace(pool, args.served_requests, seed=workloads.SEED_SERVED, rate=None)
    V.serve(sat_trace, arena, table)
    runs = {V.GROUP_AUTO: [], V.GROUP_MIXED: [], V.GROUP_BY_TREE: []}
    for _ in range(2):
        for pol in runs:
            runs[pol].append(V.summarize(V.serve(sat_trace, arena, table, grouping=pol), sat_meta))
    best = {pol: max(r, key=lambda s: s["throughput_rps"]) for pol, r in runs.items()}
    sat = best[V.GROUP_MIXED]
    out["saturation"] = sat
    out["saturation_by_grouping"] = {
        name: {"best": best[pol], "runs_rps": [r["throughput_rps"] for r in runs[pol]]}
        for name, pol in (("auto", V.GROUP_AUTO), ("always_mixed", V.GROUP_MIXED),
                          ("always_by_tree", V.GROUP_BY_TREE))}
    rate_sat = sat["throughput_rps"]
    levels = {}
    for frac in (0.25, 0.5, 0.75, 0.9):
        trace, meta = V.make_trace(pool, args.served_requests, seed=workloads.SEED_SERVED + int(100 * frac),
                                   rate=frac * rate_sat)
        levels[str(frac)] = V.summarize(V.serve(trace, arena, table), meta)
        log("bench: served at %.2f of saturation: %s" % (frac, levels[str(frac)]))
    out["poisson"] = levels
    # the same stream with every request in binary64
    trace, meta = V.make_trace(pool, args.served_requests, seed=workloads.SEED_SERVED + 50, rate=0.5 * rate_sat,
                               fp64_only=True, mix=(("f64", 1.0),))
    out["poisson_0.5_all_f64"] = V.summarize(V.serve(trace, arena, table), meta)
    # the 0.9 stream under the other grouping policies (the levels above use
    # one mixed-tree launch per element type)
    trace, meta = V.make_trace(pool, args.served_requests, seed=workloads.SEED_SERVED + 90, rate=0.9 * rate_sat)
    out["poisson_0.9_by_grouping"] = {
        name: V.summarize(V.serve(trace, arena, table, grouping=pol), meta)
        for name, pol in (("auto", V.GROUP_AUTO), ("always_by_tree", V.GROUP_BY_TREE))}
    if not args.no_parity:
        out["parity"] = served_parity(V, pool, arena, table, 0.5 * rate_sat, args.served_parity_requests)
        out["served_parity_ok"] = out["parity"]["ok"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = served_cpu_baseline(V, meta)
    del pool, arena, table
    torch.cuda.empty_cache()
    return out


def served_cpu_baseline(V, meta, budget_elems: int = 50_000_000):
    """The oracle serving the same request mix on the host's cores, one
    request after the other (throughput only): the first requests of a
    stream of the served mix (same trees, lengths and types), up to
    `budget_elems` elements, each evaluated on host operands of its length
    and type (uniform [-1, 1), seeded) with every thread this process may
    use."""
    import numpy as np

    import oracle
    from paper_1109_1264_amd import salt, workloads

    cat = dict(salt.salt_catalogue())
    sample, total = [], 0
    for m in meta:
        if total + m[2] > budget_elems:
            break
        sample.append(m)
        total += m[2]
    threads = host_threads()
    log("bench: served CPU baseline, %d requests, %d elements, %d threads" % (len(sample), total, threads))
    ops = [workloads.uniform(m[2], m[1], 7000 + i, len(m[3])) for i, m in enumerate(sample)]
    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        for m, o in zip(sample, ops):
            oracle.eval_program(cat[m[0]], o, [m[4]], m[1])
        t = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    nbytes = float(V.request_bytes(sample).sum())
    return {"value": round(len(sample) / t, 1), "unit": "requests/s", "GBps": round(nbytes / t / 1e9, 3),
            "cores": threads, "kind": "oracle",
            "sample": "%d requests (%d elements) of the same trees, lengths and type mix, served one after the "
                      "other by the oracle on host operands" % (len(sample), total)}


def served_parity(V, pool, arena, table, rate, count):
    """A Poisson stream of the same workload served with kept outputs; every
    request's output is compared bit for bit with the oracle's evaluation of
    its tree on host copies of its operands, at 4096 random elements plus its
    first and last 1024 (all elements when it is shorter)."""
    import numpy as np
    import torch

    import oracle
    from paper_1109_1264_amd import salt, workloads

    log("bench: served parity, %d requests against the oracle" % count)
    trace, meta = V.make_trace(pool, count, seed=workloads.SEED_SERVED + 77, rate=rate)
    res = V.serve(trace, arena, table, keep_outputs=True)
    torch.cuda.synchronize()
    cat = dict(salt.salt_catalogue())
    bits = {"f64": np.uint64, "f32": np.uint32, "bf16": np.uint16}
    rng = np.random.Generator(np.random.PCG64(workloads.SEED_SERVED + 78))
    bad, elems = [], 0
    for i, (r, m) in enumerate(zip(res, meta)):
        tree, dt, n, offs, alpha = m
        if r.status != 0:
            bad.append(i)
            continue
        idx = None if n <= 4096 + 2048 else np.unique(np.concatenate(
            [rng.integers(0, n, 4096), np.arange(1024), np.arange(n - 1024, n)]))
        ops, got = V.request_host_bits(pool, arena, r, m, idx)
        want = oracle.eval_program(cat[tree], ops, [alpha], dt)
        if not np.array_equal(got.view(bits[dt]), want.view(bits[dt])):
            bad.append(i)
        elems += n if idx is None else len(idx)
    combos = sorted({"%s/%s" % (m[0], m[1]) for m in meta})
    return {"requests": count, "elements_checked": int(elems), "tree_dtype_pairs": len(combos),
            "max_n": int(max(m[2] for m in meta)), "mismatched_requests": bad[:20],
            "what": "served outputs (kept) vs the oracle on host copies of each request's operands, "
                    "bit for bit, 4096 random elements + first/last 1024 per request",
            "ok": not bad}


def sum_prog(k: int) -> list:
    """Postfix program of op0 + op1 + ... + op(k-1), left to right."""
    import paper_1109_1264_amd.salt as salt

    p = [salt.token(salt.LOAD, 0)]
    for j in range(1, k):
        p += [salt.token(salt.LOAD, j), salt.token(salt.ADD)]
    return p


def launch_only(args) -> None:
    """Launch the named kernels --steps times each and print nothing else
    (for counter collection under rocprofv3). Each spec is
    kind:dtype:log2n, kind one of dot, nrm2 (whole call), dot1, nrm21 (pass 1
    only), rsum3, rsum5 (nrm2 of the sum of 3 or 5 operands on its run-time
    compiled kernel: 3 or 5 read streams and no write), tree5, fig1, axpy, t4, t5, copy (catalogue trees
    writing a fresh output). Inputs cycle through enough copies that each
    launch reads past the 256 MiB last-level cache."""
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    cat = dict(salt.salt_catalogue())
    codes = {"f64": salt.F64, "f32": salt.F32, "bf16": salt.BF16, "f16": salt.F16}
    for spec in args.launch_only.split(","):
        kind, dt, l2 = spec.split(":")
        n = 1 << int(l2)
        es = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[dt]
        loads = {"dot": 2, "dot1": 2, "nrm2": 1, "nrm21": 1, "rsum3": 3, "rsum5": 5}.get(kind)
        if loads is None:
            loads = 1 + max(t >> 8 for t in cat[kind] if t & 0xFF == salt.LOAD)
        set_bytes = loads * es * n
        sets = max(2, min(8, -(-(1 << 30) // set_bytes)))
        ops = [workloads.uniform_device(n, dt, workloads.sweep_seed(n) + k, loads) for k in range(sets)]
        code = codes[dt]
        ws = salt.workspace(n, code)
        part = torch.empty(max(1, salt.salt_reduce_workspace_bytes(n, code) // 8), dtype=torch.float64,
                           device="cuda")
        out = torch.empty(n, dtype=ops[0][0].dtype, device="cuda") if kind in cat else None
        if kind in ("rsum3", "rsum5"):
            salt.salt_jit_compile_reduce(sum_prog(loads), None, loads, 0, code)  # every launch compiled
        for s in range(args.steps):
            v = ops[s % sets]
            if kind == "dot":
                salt.salt_dot(v[0], v[1], ws=ws)
            elif kind == "nrm2":
                salt.salt_nrm2(v[0], ws=ws)
            elif kind == "dot1":
                salt.salt_reduce_partials(salt.MODE_DOT, v[0], v[1], partials=part)
            elif kind == "nrm21":
                salt.salt_reduce_partials(salt.MODE_NRM2, v[0], partials=part)
            elif kind in ("rsum3", "rsum5"):
                salt.salt_nrm2_expr(sum_prog(loads), v, [], ws=ws)
            else:
                salt.salt_eval(cat[kind], v, [1.25], out)
        torch.cuda.synchronize()
        log("bench: launched %s x%d" % (spec, args.steps))
        del ops, ws, part, out
        torch.cuda.empty_cache()


def mix_ceilings(out: dict) -> None:
    """The read/write-mix ceilings of the batched and served workloads, from
    the stream references the mix section measured on this GPU: the batched
    tree reads 3 operands and writes 1 (its dot reads nothing more); a served
    request of a tree with k operands moves (k + 1) units per element and
    the trees are drawn uniformly, so the served ceiling is the byte-weighted
    harmonic mean of the (k, 1) references."""
    from paper_1109_1264_amd import serve as V

    refs = {(r[0], r[1]): r[3] for r in out["mix"]["rows"]}
    b = out.get("batched")
    if b and (3, 1) in refs:
        b["mix_ceiling_GBps"] = refs[(3, 1)]
        b["graph_frac_of_mix_ceiling"] = round(b["graph_GBps"] / refs[(3, 1)], 4)
    sm = out.get("served_summary")
    if sm:
        w = [(V.tree_loads(t) + 1, V.tree_loads(t)) for t in V.TREES]
        if all((k, 1) in refs for _, k in w):
            ceil = sum(u for u, _ in w) / sum(u / refs[(k, 1)] for u, k in w)
            sm["mix_ceiling_GBps"] = round(ceil, 1)
            sm["saturation_frac_of_mix_ceiling"] = round(sm["saturation_GBps"] / ceil, 4)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--sections", default="main,mix,sweep,fusion,precision,blas1,vendor,batched,served")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--cpu-log2n", type=int, default=26)
    ap.add_argument("--pool-gb", type=int, default=64)
    ap.add_argument("--served-requests", type=int, default=10000)
    ap.add_argument("--served-parity-requests", type=int, default=1000)
    ap.add_argument("--kernels-only", default=None,
                    help="comma list of tree5,axpy,dot,nrm2,copy: launch only these, --steps times "
                         "each, and print nothing (for counter collection)")
    ap.add_argument("--launch-only", default=None,
                    help="comma list of kind:dtype:log2n (see launch_only): launch only these, --steps "
                         "times each, and print nothing (for counter collection)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(element-wise work shards by index range and dot/nrm2 need one 8-byte "
              "combine; see the design notes). Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    torch.cuda.set_device(0)
    out = {"metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    sections = args.sections.split(",")
    if args.kernels_only:
        section_main(args, out)
        return 0
    if args.launch_only:
        launch_only(args)
        return 0
    if "main" in sections:
        section_main(args, out)
    if "mix" in sections:
        out["mix"] = section_mix(args)
        ref51 = [r for r in out["mix"]["rows"] if r[0] == 5 and r[1] == 1][0]
        if out.get("roofline"):
            ach = out["roofline"]["achieved"]
            out["roofline"]["mix_ceiling"] = {
                "GBps": ref51[3], "frac_of_peak": round(ref51[3] / HBM_PEAK_GBPS, 4),
                "what": "plain 5-read 1-write stream reference on the same GPU, one dispatch per call (bench "
                        "section mix); the tree's call runs as chunked dispatches that keep its persistent "
                        "grid in step, which this one-dispatch reference does not bound"}
            out["roofline"]["frac_of_mix_ceiling"] = round(ach / ref51[3], 4)
    if "sweep" in sections:
        out["sweep"] = section_sweep(args)
    if "fusion" in sections:
        out["fusion"] = section_fusion(args)
    if "precision" in sections:
        out["precision"] = section_precision(args)
    if "blas1" in sections:
        out["blas1"] = section_blas1(args)
    if "vendor" in sections:
        out["vendor_blas"] = section_vendor(args)
    if "batched" in sections:
        out["batched"] = section_batched(args)
    if "served" in sections:
        out["served"] = section_served(args)
        sv = out["served"]
        out["served_summary"] = {
            "saturation_rps": sv["saturation"]["throughput_rps"], "saturation_GBps": sv["saturation"]["GBps"],
            "p50_ms_at_0.9": sv["poisson"]["0.9"]["p50_ms"], "p99_ms_at_0.9": sv["poisson"]["0.9"]["p99_ms"],
            "p50_ms_at_0.5": sv["poisson"]["0.5"]["p50_ms"], "p99_ms_at_0.5": sv["poisson"]["0.5"]["p99_ms"],
            "served_parity_ok": sv.get("served_parity_ok")}
    if "mix" in out:
        mix_ceilings(out)
    if not args.no_cpu_baseline and "main" in sections:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(args.cpu_log2n)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
