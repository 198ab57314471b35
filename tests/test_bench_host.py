"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
work per launch that the roofline divides by the measured time, and the
measured-traffic lines it reads from the rocprofv3 summaries."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    # the build has no multi-GPU path: --gpus N > 1 exits with a message
    # before touching torch or a device
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_of_the_grid_kernels():
    # sweep: p read once (every element), q written once (interior); copy:
    # interior read once and written once -- at the large grid these are
    # the figures quoted in the profiles
    I, J, K = 513, 513, 1025
    interior = (I - 2) * (J - 2) * (K - 2)
    assert bench.stencil_bytes(I, J, K) == 4 * I * J * K + 4 * interior == 2147500032
    assert bench.copy_interior_bytes(I, J, K) == 8 * interior == 2137014264
    assert bench.stencil_bytes(3, 3, 3) == 4 * 27 + 4 and bench.copy_interior_bytes(3, 3, 3) == 8


def test_large_work_per_launch():
    w = bench.large_work({"I": 513, "J": 513, "K": 1025, "N": 8192})
    assert w["gemm"][:4] == (2.0 * 8192 ** 3, "TFLOP/s", "mfma", 157.3)
    assert w["gemm_bf16"][:4] == (2.0 * 8192 ** 3, "TFLOP/s", "mfma", 2500.0)
    assert w["stencil19"][0] == bench.stencil_bytes(513, 513, 1025) and w["stencil19"][2] == "hbm"


def test_roofline_entry_arithmetic():
    live = {"avg_us": 400.0, "launches": 10, "total_ms": 4.0}
    e = bench.roof_entry("gemm", (8e9, "TFLOP/s", "mfma", 157.3), live, "w")
    assert e["achieved"] == pytest.approx(20.0) and e["frac"] == pytest.approx(20.0 / 157.3, abs=1e-4)
    assert e["traffic"] is None and e["flops_per_launch"] == 8e9


def test_measured_traffic_lines():
    # every `traffic:` line of profiles/ names a kernel kind whose sources
    # bench.py knows; measured_traffic returns the line's bytes while the
    # kind's sources are unchanged, else None
    pat = re.compile(r"^traffic: (\S+) (\S+) (\d+) sources ([0-9a-f]{16})\s*$")
    seen = 0
    pdir = os.path.join(ROOT, "profiles")
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                if not line.startswith("traffic:"):
                    continue
                m = pat.match(line.strip())
                assert m, line
                kind, workload, nbytes, sha = m.group(1), m.group(2), int(m.group(3)), m.group(4)
                assert kind in bench.KERNEL_SOURCES
                got = bench.measured_traffic(kind, workload)
                assert got == (nbytes if sha == bench.sources_sha(kind) else None)
                seen += 1
    assert seen >= 2
    assert bench.measured_traffic("stencil19", "no_such_workload") is None


def test_nan_none():
    assert bench.nan_none(float("nan")) is None
    assert bench.nan_none(1.23456, 2) == 1.23
