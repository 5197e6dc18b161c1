"""The benchmark's command-line contract and its CPU-baseline leg, on the CPU:
more than one GPU is refused with a message and exit status 2, and the
baseline record names its unit, the threads it used and the host."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_cpu_baseline_record():
    sys.path.insert(0, ROOT)
    import bench

    rec = bench.cpu_baseline(12, reps=1)
    assert rec["kind"] == "oracle" and rec["unit"] == "GB/s"
    # all the threads the process may use, and a one-thread figure beside them
    assert rec["cores"] == bench.host_threads() >= 1
    assert rec["value"] > 0 and rec["seconds_per_step"] > 0
    assert rec["one_thread"]["value"] > 0
    assert rec["dot2_reference_seconds"]["dot_and_nrm2"] > 0
    assert "n=2^12" in rec["sample"]
    assert rec["host"]["logical_cpus"] == os.cpu_count()
    json.dumps(rec)  # one JSON line


def test_traffic_only_for_the_profiled_kernel_source(tmp_path):
    """The counter-derived traffic is reported only while the committed
    counter summary was taken on the current tree-kernel source."""
    sys.path.insert(0, ROOT)
    import bench

    with open(bench.PROFILE_PMC) as fh:
        prof = json.load(fh)
    got = bench.traffic_from_profile(prof["n"])
    from paper_1109_1264_amd import salt as S

    same_split = S.salt_eval_chunking(5, prof["n"], S.F64)[1] == prof["dispatches_per_launch"]
    if prof["kernel_source_hash"] == bench.kernel_source_hash() and same_split:
        assert got == prof["traffic_bytes_per_launch"]
    else:
        assert got is None
    # a record taken with another split of the call is not used
    other = dict(prof, dispatches_per_launch=prof["dispatches_per_launch"] + 1)
    alt = os.path.join(str(tmp_path), "pmc.json")
    with open(alt, "w") as fh:
        json.dump(other, fh)
    saved = bench.PROFILE_PMC
    bench.PROFILE_PMC = alt
    try:
        assert bench.traffic_from_profile(prof["n"]) is None
    finally:
        bench.PROFILE_PMC = saved


def test_traffic_is_derived_from_request_counts():
    """The committed traffic figure is the request counts times their sizes
    (128-byte reads, 64- or 32-byte writes), not a factor fitted to another
    kernel, and it matches the algorithmic bytes of the tree kernel."""
    sys.path.insert(0, ROOT)
    import bench

    with open(bench.PROFILE_PMC) as fh:
        prof = json.load(fh)
    c = prof["counters_per_launch"]
    rd = 128 * (c["TCC_EA0_RDREQ_sum"] - c["TCC_EA0_RDREQ_32B_sum"]) + 32 * c["TCC_EA0_RDREQ_32B_sum"]
    wr = 64 * c["TCC_EA0_WRREQ_64B_sum"] + 32 * (c["TCC_EA0_WRREQ_sum"] - c["TCC_EA0_WRREQ_64B_sum"])
    assert prof["read_bytes_per_launch"] == rd and prof["write_bytes_per_launch"] == wr
    assert prof["traffic_bytes_per_launch"] == rd + wr
    assert abs(prof["traffic_bytes_per_launch"] / prof["algorithmic_bytes_per_launch"] - 1) < 1e-4
    assert prof["algorithmic_bytes_per_launch"] == 48 * prof["n"]


def test_served_cpu_baseline_record():
    """The oracle's throughput on a served-like request mix: a bounded sample,
    its thread count and the requests/s unit."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1109_1264_amd import serve as V

    meta = [("fig1", "f32", 5000, [0, 64, 128], 1.5), ("t5", "bf16", 3000, [0] * 6, 0.75),
            ("axpy", "f64", 4000, [0, 64], 1.25), ("tree5", "f32", 10 ** 9, [0] * 5, 1.0)]
    rec = bench.served_cpu_baseline(V, meta, budget_elems=20000)
    assert rec["kind"] == "oracle" and rec["unit"] == "requests/s" and rec["value"] > 0
    assert rec["cores"] == bench.host_threads()
    assert rec["sample"].startswith("3 requests (12000 elements)")


def test_mix_ceilings_of_batched_and_served():
    """The batched workload's ceiling is the 3-read 1-write reference; the
    served one is the byte-weighted harmonic mean of its trees' (k, 1)
    references (k + 1 units per element, trees drawn uniformly)."""
    sys.path.insert(0, ROOT)
    import bench

    rows = [[k, 1, 0.0, 8000.0 - 500.0 * k, 0.0, "", 0.0, 0.0, 0.0] for k in range(1, 7)]
    out = {"mix": {"rows": rows}, "batched": {"graph_GBps": 5000.0},
           "served_summary": {"saturation_GBps": 5000.0}}
    bench.mix_ceilings(out)
    assert out["batched"]["mix_ceiling_GBps"] == 6500.0
    assert out["batched"]["graph_frac_of_mix_ceiling"] == round(5000.0 / 6500.0, 4)
    # fig1 (3 operands), axpy (2), tree5 (5), t4 (4), t5 (6)
    units = {3: 4, 2: 3, 5: 6, 4: 5, 6: 7}
    want = sum(units.values()) / sum(u / (8000.0 - 500.0 * k) for k, u in units.items())
    assert abs(out["served_summary"]["mix_ceiling_GBps"] - want) < 0.06
    assert out["served_summary"]["saturation_frac_of_mix_ceiling"] == round(
        5000.0 / out["served_summary"]["mix_ceiling_GBps"], 4)
