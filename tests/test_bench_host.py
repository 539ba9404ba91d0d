"""Host logic of bench.py, no GPU: the algorithmic bytes each workload's roofline is
priced with, the matcher that takes a launch's measured HBM traffic from a committed
counter summary only while the kernel sources it was taken on are unchanged, and the
refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2008_04356_amd import workloads as W  # noqa: E402


# Totals written out from the per-point figures: every mortar point (a face point of
# either side, 2 F P per interface) reads its inputs once and writes its 5 outputs once;
# Navier-Stokes reads 5 states and 15 gradients (25 values, 100 B in FP32, 200 B in
# FP64), Euler 5 states (10 values, 40 B / 80 B); per-point metrics add 4 values at each
# static face point (16 B / 32 B).
@pytest.mark.parametrize("idx, precision, expected", [
    (1, W.FP64, 2 * 8 * 8 * 16 * 80),                                   # 163,840
    (2, W.FP32, 2 * 128 * 64 * 36 * 100),                               # 58,982,400
    (3, W.FP32, 2 * 512 * 64 * 64 * 100 + 512 * 64 * 64 * 16),          # 452,984,832
    (3, W.FP64, 2 * 512 * 64 * 64 * 200 + 512 * 64 * 64 * 32),          # 905,969,664
    (4, W.FP32, 2 * (320 * 125 * 64 + 256 * 72 * 36 + 64 * 32 * 16) * 100
     + (320 * 125 * 64 + 256 * 72 * 36) * 16),                          # 702,840,832
    (5, W.FP32, 2 * 256 * 256 * 100 * 40),                              # 524,288,000
])
def test_algorithmic_bytes_per_workload(idx, precision, expected):
    specs, _ = W.config(idx, precision=precision)
    assert sum(bench.algorithmic_bytes(s) for s in specs) == expected


def test_algorithmic_bytes_of_the_documented_workloads():
    # the figures the profiles and the roofline quote
    specs, _ = W.config(4)
    assert sum(bench.algorithmic_bytes(s) for s in specs) == 702_840_832
    assert sum(s.mortar_points for s in specs) == 6_512_640
    specs, _ = W.config(2)
    assert bench.algorithmic_bytes(specs[0]) == 58_982_400


def _profile(tmp_path, lines):
    p = tmp_path / "summary.md"
    p.write_text("# counter summary\n\nsome text\n" + "\n".join(lines) + "\n")
    return str(p)


def test_measured_traffic_matches_launch_and_source_hash(tmp_path, monkeypatch):
    good = bench.sources_sha256(["mortar_internal.h"])
    bad = "0" * 64
    path = _profile(tmp_path, [
        f"launch variant=2 tile_len=15 grid=0 traffic=111 sources=mortar_internal.h sha256={good}",
        f"launch variant=2 tile_len=15,15,10 grid=0 traffic=222 sources=mortar_internal.h sha256={good}",
        f"launch variant=0 tile_len=20 grid=0 traffic=333 sources=mortar_internal.h sha256={bad}",
    ])
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {2: path, 4: path})

    def tun(v, tiles, g=0):
        return [{"variant": v, "tile_len": t, "grid": g} for t in tiles]

    assert bench.measured_traffic(2, "fp32", tun(2, [15])) == 111
    assert bench.measured_traffic(4, "fp32", tun(2, [15, 15, 10])) == 222
    # another tile list, grid or variant: no line for that launch
    assert bench.measured_traffic(4, "fp32", tun(2, [15, 15, 15])) is None
    assert bench.measured_traffic(2, "fp32", tun(2, [15], g=64)) is None
    assert bench.measured_traffic(2, "fp32", tun(3, [15])) is None
    # the sources changed since the counters were taken
    assert bench.measured_traffic(2, "fp32", tun(0, [20])) is None
    # only FP32 launches and workloads with a summary
    assert bench.measured_traffic(2, "bf16", tun(2, [15])) is None
    assert bench.measured_traffic(3, "fp32", tun(2, [15])) is None
    assert bench.measured_traffic(2, "fp32", []) is None


def test_measured_traffic_malformed_line(tmp_path, monkeypatch):
    path = _profile(tmp_path, ["launch variant=2 tile_len=15 grid=0 traffic=notanumber"])
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {2: path})
    assert bench.measured_traffic(2, "fp32", [{"variant": 2, "tile_len": 15, "grid": 0}]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
