"""Benchmark of the SALT hot path on one MI355X.

One step = one pass of the hot path over one batch of HBM-resident synthetic
vectors (BLAS-1 sweep at its largest size, n = 2^28, binary64):
    d = a*b + c*e - f      (fused 5-operand tree, salt_eval)
    d = alpha*a + d        (salt_axpy, in place)
    dot(a, b)              (salt_dot)
    nrm2(c)                (salt_nrm2)
`value` = algorithmic bytes of the step (inputs read once + outputs written
once) / wall time per step, in GB/s. Per-kernel durations come from HIP
events recorded on the launch stream inside the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--log2n 28]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "achieved HBM GB/s (% of peak) on fused vector exprs; served p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("eval.hip", "device.hpp", "expr.hpp"):
        with open(os.path.join(ROOT, "paper_1109_1264_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(n_elems: int):
    """HBM bytes per launch of the tree kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "pmc_tree5_f64_n2p28.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("n") != n_elems:
        return None
    return d.get("traffic_bytes_per_launch")


def cpu_baseline(log2n_sample: int, reps: int = 3):
    """The oracle (plain C, one thread) on a bounded sample of the step."""
    import numpy as np

    import oracle
    from paper_1109_1264_amd import workloads

    n = 1 << log2n_sample
    a, b, c, e, f = workloads.uniform(n, "f64", workloads.sweep_seed(n), 5)
    alpha = workloads.alpha(workloads.sweep_seed(n))
    tree5 = [1, (1 << 8) | 1, 5, (2 << 8) | 1, (3 << 8) | 1, 5, 3, (4 << 8) | 1, 4]
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        d = oracle.eval_program(tree5, [a, b, c, e, f], [], "f64")
        d = oracle.axpy(alpha, a, d, "f64")
        oracle.dot2(a, b)
        oracle.nrm2(c)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return {"value": round(96.0 * n / t / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "one step of the same hot path (tree eval, axpy, Dot2 dot, Dot2 nrm2) on n=2^%d "
                      "binary64 elements, median of %d, single-threaded plain C" % (log2n_sample, reps),
            "seconds_per_step": round(t, 4)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--cpu-log2n", type=int, default=26)
    ap.add_argument("--kernels-only", default=None,
                    help="comma list of tree5,axpy,dot,nrm2,copy: launch only these, --steps times "
                         "each, and print nothing else (for counter collection)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(element-wise work shards by index range and dot/nrm2 need one 8-byte "
              "combine; see the design notes). Run with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1109_1264_amd.salt as salt
    from paper_1109_1264_amd import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
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
        else:
            salt.salt_nrm2(c, result=r_nrm, ws=ws)

    def step(events=None):
        for k in names:
            if events is not None:
                events[k][0].record()
            launch(k)
            if events is not None:
                events[k][1].record()

    if args.kernels_only:
        for k in args.kernels_only.split(","):
            for _ in range(args.steps):
                if k == "copy":
                    salt.salt_eval(copy, [a], [], d)
                else:
                    launch(k)
            torch.cuda.synchronize()
            log("bench: ran %s x%d" % (k, args.steps))
        return 0

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: wall clock over K steps, events around every launch
    ev = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in names}
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    per = {k: float(np.mean([ev[s][k][0].elapsed_time(ev[s][k][1]) for s in range(args.steps)])) for k in names}
    step_bytes = sum(bytes_per_elem.values()) * n
    value = step_bytes / (wall / args.steps) / 1e9

    # copy kernel (d = a) as the attainable-bandwidth ceiling, same machinery
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for s0, s1 in cev:
        s0.record()
        salt.salt_eval(copy, [a], [], d)
        s1.record()
    torch.cuda.synchronize()
    copy_ms = float(np.mean([s0.elapsed_time(s1) for s0, s1 in cev[2:]]))
    copy_gbps = 16.0 * n / (copy_ms * 1e-3) / 1e9

    kernels = {k: {"avg_ms": round(per[k], 4), "GBps": round(bytes_per_elem[k] * n / (per[k] * 1e-3) / 1e9, 1),
                   "bytes_per_elem": bytes_per_elem[k]} for k in names}
    dom = "tree5"
    achieved = bytes_per_elem[dom] * n / (per[dom] * 1e-3) / 1e9
    traffic = traffic_from_profile(n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "k_eval_tree<tree5, f64> (d = a*b + c*e - f)",
                "algorithmic_bytes_per_launch": bytes_per_elem[dom] * n}

    parity = None
    if not args.no_parity:
        parity = check_parity(n, a, b, c, e, f, d, r_dot, r_nrm, ws, tree5)

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(args.cpu_log2n)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "BLAS-1 sweep, largest size: d=a*b+c*e-f, y=alpha*x+y, dot(x,y), nrm2(x); "
                               "binary64, n=2^%d, uniform[-1,1) operands resident in HBM" % args.log2n,
                   "n": n, "seed": seed, "alpha": alpha, "step_bytes": step_bytes},
        "pct_of_hbm_peak": round(100.0 * value / HBM_PEAK_GBPS, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "copy_ceiling": {"avg_ms": round(copy_ms, 4), "GBps": round(copy_gbps, 1),
                         "pct_of_hbm_peak": round(100 * copy_gbps / HBM_PEAK_GBPS, 2)},
        "parity": parity,
    }
    print(json.dumps(out), flush=True)
    return 0


def check_parity(n, a, b, c, e, f, d, r_dot, r_nrm, ws, tree5):
    """Sampled bit-exact check of the tree kernel and full-length tolerance
    checks of dot / nrm2 against the oracle, at the benchmarked size."""
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
    return {"tree5_sampled_bit_exact": eval_ok, "samples": int(len(idx)),
            "dot_rel_err": dot_err, "nrm2_rel_err": nrm_err, "tol": 1e-13,
            "ok": bool(eval_ok and dot_err <= 1e-13 and nrm_err <= 1e-13)}


if __name__ == "__main__":
    sys.exit(main())
