"""The serving loop's host logic (csrc/server.hip) on the CPU.

The loop is compiled for the host only and linked with an emulation of its
device side (``tests/server_emu/emu.cpp``): streams run their queued copies,
launches and event records in order at random moments, so every seed gives a
different interleaving of completions. Each emulated launch checks its
descriptor table, its (item, tile) list (as a whole when the loop splits a
long list over several launches) and every element range its tiles
touch against the operand pool and the output arena, and that no output
overlaps the output of a batch the host has not yet seen complete. Traces are
the served benchmark's (same generator and seeds) with addresses of a pool
that exists only as numbers. A copy of the loop with a planted mistake (a
slot released when its first group finishes instead of its last) must fail
the same checks."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

from paper_1109_1264_amd import serve as V
from paper_1109_1264_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1109_1264_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = ["-x", "hip", "--cuda-host-only", "-O1", "-std=c++17", "-fPIC",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")


class NumberPool:
    """The served benchmark's pool layout (64 GB, the dtype mix), as addresses only."""

    def __init__(self, total_bytes, mix=V.MIX):
        self.base, self.n, self.es = {}, {}, {}
        addr = 0x100000000000
        for name, frac in mix:
            es = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[name]
            n = int(total_bytes * frac) // es // 4096 * 4096
            self.base[name], self.n[name], self.es[name] = addr, n, es
            addr += (n * es + (1 << 30)) // (1 << 21) * (1 << 21)

    def elems(self, d):
        return self.n[d]

    def ptr(self, d, off):
        return self.base[d] + off * self.es[d]


def build(tmp, server_src):
    objs = []
    for src, name in ((server_src, "server.o"), (os.path.join(ROOT, "tests", "server_emu", "emu.cpp"), "emu.o")):
        out = os.path.join(tmp, name)
        subprocess.check_call([HIPCC, *FLAGS, "-c", src, "-o", out])
        objs.append(out)
    exe = os.path.join(tmp, "emu")
    subprocess.check_call(["g++", "-pie", *objs, "-o", exe])
    return exe


@pytest.fixture(scope="module")
def setup(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("server_emu"))
    pool = NumberPool(64 << 30)
    with open(os.path.join(tmp, "pool.txt"), "w") as fh:
        for name in pool.base:
            fh.write("%s %d %d %d\n" % (name, pool.base[name], pool.n[name], pool.es[name]))
    S = workloads.SEED_SERVED
    traces = {}
    for name, count, seed, rate, kw in (("warm", 2000, S + 999, None, {}), ("saturation", 6000, S, None, {}),
                                        ("poisson", 4000, S + 90, 150000.0, {}),
                                        ("f64", 3000, S + 50, 80000.0, dict(fp64_only=True, mix=(("f64", 1.0),)))):
        tr, _ = V.make_trace(pool, count, seed=seed, rate=rate, **kw)
        path = os.path.join(tmp, "trace_%s.bin" % name)
        with open(path, "wb") as fh:
            fh.write(bytes(tr))
        traces[name] = path
    return tmp, build(tmp, os.path.join(CSRC, "server.hip")), traces


def run(exe, tmp, trace, arena_gb, p, seed, max_batch=512, streams=4, depth=2, grouping=0, range_bytes=0):
    return subprocess.run([exe, os.path.join(tmp, "pool.txt"), trace, str(arena_gb), str(p), str(seed),
                           str(max_batch), str(streams), str(depth), str(grouping), str(range_bytes)],
                          capture_output=True, text=True, timeout=300)


@pytest.mark.parametrize("grouping", [0, 1, 2])
@pytest.mark.parametrize("trace", ["warm", "saturation", "poisson", "f64"])
def test_loop_tables_tiles_and_addresses(setup, trace, grouping):
    tmp, exe, traces = setup
    for arena_gb, p, seed, mb, ns, dp in ((32, 0.3, 1, 512, 4, 2), (8, 0.05, 2, 512, 4, 2), (32, 1.0, 3, 128, 8, 4),
                                          (4, 0.02, 4, 2048, 2, 1)):
        r = run(exe, tmp, traces[trace], arena_gb, p, seed, mb, ns, dp, grouping)
        assert r.returncode == 0, (trace, arena_gb, p, seed, r.stdout, r.stderr[-2000:])


@pytest.mark.parametrize("range_bytes", [16 << 20, 64 << 20, -1])
def test_split_tile_lists(setup, range_bytes):
    """Long tile lists run as consecutive ranges (down to 16 MiB per operand,
    so most large groups split): every tile of every group runs exactly
    once, all groups complete, and the other checks hold; -1 never splits."""
    tmp, exe, traces = setup
    for trace, seed in (("saturation", 5), ("poisson", 6)):
        r = run(exe, tmp, traces[trace], 32, 0.3, seed, 512, 4, 2, 0, range_bytes)
        assert r.returncode == 0, (trace, range_bytes, r.stdout, r.stderr[-2000:])
        split = int(r.stdout.split("launches (")[1].split(" of split")[0])
        assert (split > 0) == (range_bytes > 0), r.stdout


def test_planted_early_release_is_caught(setup, tmp_path):
    tmp, _, traces = setup
    src = open(os.path.join(CSRC, "server.hip")).read()
    good = "hipEventQuery(sl.ev[sl.n_groups - 1])"
    assert good in src
    mutant = tmp_path / "server_mutant.hip"
    mutant.write_text(src.replace(good, "hipEventQuery(sl.ev[0])"))
    exe = build(str(tmp_path), str(mutant))
    r = run(exe, tmp, traces["saturation"], 32, 0.05, 1)
    assert r.returncode == 1 and "overlaps a live output" in r.stderr, (r.stdout, r.stderr[-500:])
