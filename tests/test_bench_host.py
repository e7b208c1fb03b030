"""Host-side arithmetic of bench.py (no GPU): the one-GPU guard, the
algorithmic byte counts behind the roofline objects, the roofline
arithmetic, and the reading of the committed counter summaries."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_arc_discovery_bytes():
    # 8 B per row entry (column entry + stamp), 16 B per member (two row
    # offsets), 4 B per probed out-list entry
    st = {"k4_main_kind": 6, "k4_main_entries": 1000, "k4_main_nbrs": 300, "k4_main_pairs": 50000}
    assert bench.main_kernel_bytes(st) == 8 * 1000 + 16 * 300 + 4 * 50000
    # the stage figure adds every member's stamp and degree update (20 B)
    assert bench.k4_bytes(dict(st, m=10**6, s2=0), 4) == 8 * 1000 + 16 * 300 + 4 * 50000 + 20 * 300


def test_other_main_kernel_bytes():
    assert bench.main_kernel_bytes({"k4_main_kind": 3, "k4_main_pairs": 10, "k4_main_nbrs": 2}) == 16 * 10 + 24 * 2
    assert bench.main_kernel_bytes({"k4_main_kind": 1, "k4_main_pairs": 10, "k4_main_nbrs": 2}) == 24 * 10 + 16 * 2
    assert bench.main_kernel_bytes({"k4_main_kind": 2, "k4_main_pairs": 10, "k4_main_nbrs": 2}) == 4 * 10 + 20 * 2
    assert bench.k4_bytes({"m": 7, "k4_main_kind": 1}, 2) == 32 * 7
    assert bench.k4_bytes({"m": 7, "s2": 11, "k4_main_kind": 3}, 3) == 4 * 11 + 24 * 7


def test_tail_engine_bytes():
    st = {"k4_tail_pairs": 1000, "k4_tail_vertices": 10, "k4_tail_grid_rounds": 3}
    assert bench.tail_kernel_bytes(st) == 4 * 1000 + 40 * 10 + 18 * 10 * 3


def test_hbm_roofline_arithmetic():
    # 100 launches moving 2e8 B in 50 ms: 2e6 B in 0.5 ms a launch = 4 GB/s
    r = bench.roof("k_none", "no_workload", 50.0, 100, 2e8)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["bytes_per_launch"] == pytest.approx(2e6)
    assert r["ms_per_launch"] == pytest.approx(0.5)
    assert r["achieved"] == pytest.approx(4.0)
    assert r["frac"] == pytest.approx(4.0 / 8000.0)
    assert r["traffic"] is None                     # no summary for this kernel


def test_alu_roofline_arithmetic():
    # 10 launches counting 1e9 words in 100 ms: 1e8 words in 10 ms = 0.01 Tword/s
    r = bench.roof_alu("k_none", 100.0, 10, 1e9)
    assert r["bound"] == "alu"
    assert r["peak"] == pytest.approx(256 * 64 * 2.4e9 / 4 / 1e12)
    assert r["achieved"] == pytest.approx(0.01)
    assert r["frac"] == pytest.approx(0.01 / r["peak"])


def _summary_fields(path):
    fields = {}
    for line in open(path):
        if line.startswith(("traffic_bytes_per_launch:", "kernel_source_sha256:")):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    return fields


@pytest.mark.parametrize("kernel,workload", [("k_root_edges", "rmat22_h4"), ("k_tail_engine", "chung_lu_1e6")])
def test_traffic_follows_the_measured_source(kernel, workload, tmp_path, monkeypatch):
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    fields = _summary_fields(path)
    sha = hashlib.sha256(open(bench.PEEL_SOURCE, "rb").read()).hexdigest()
    got = bench.measured_traffic(kernel, workload)
    if fields["kernel_source_sha256"] == sha:
        assert got == float(fields["traffic_bytes_per_launch"])
    else:
        assert got is None
    # any other peel source: the figure is withheld
    other = tmp_path / "peel.hip"
    other.write_text("// a different source\n")
    monkeypatch.setattr(bench, "PEEL_SOURCE", str(other))
    assert bench.measured_traffic(kernel, workload) is None


def test_no_summary_no_traffic():
    assert bench.measured_traffic("k_not_a_kernel", "rmat22_h4") is None
