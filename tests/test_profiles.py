"""The committed rocprofv3 summaries: each names the command that made it,
the command runs committed files only, and the summaries bench.py reads
carry the fields it parses."""
from __future__ import annotations

import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUMMARIES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))


def test_there_are_summaries():
    assert SUMMARIES


@pytest.mark.parametrize("path", SUMMARIES, ids=os.path.basename)
def test_summary_names_its_command(path):
    text = open(path).read()
    if os.path.basename(path).startswith("counters_"):
        # tables over the runs of a traffic summary, which hold the commands
        assert "rocprofv3" in text or "Same runs" in text
    else:
        assert "rocprofv3 --" in text
    for cmd in re.findall(r"rocprofv3 [^\n]*", text):
        if " -- " not in cmd:
            continue
        prog = cmd.split(" -- ", 1)[1]
        # the profiled program is the program itself (no launcher), and a
        # committed script when it is a file of this repository
        assert not prog.startswith(("env ", "bash ", "sh ", "taskset", "numactl"))
        assert "_work" not in prog
        for f in re.findall(r"(\S+\.py)\b", prog):
            assert os.path.exists(os.path.join(ROOT, f)), f


@pytest.mark.parametrize("path", [p for p in SUMMARIES if "traffic_bytes_per_launch" in open(p).read()],
                         ids=os.path.basename)
def test_traffic_fields(path):
    fields = {}
    for line in open(path):
        if line.startswith(("traffic_bytes_per_launch:", "kernel_source_sha256:")):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    assert float(fields["traffic_bytes_per_launch"]) > 0
    assert re.fullmatch(r"[0-9a-f]{64}", fields["kernel_source_sha256"])
    name = os.path.basename(path)
    assert name.startswith("k_") and name.endswith("_traffic.md")   # <kernel>_<workload>_traffic.md
