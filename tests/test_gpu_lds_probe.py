"""The LDS rates bench.py's heat roofline takes as the peak
(LDS_READ_B_PER_CLK, LDS_WRITE_B_PER_CLK) are what the probe measures on
this device: tests/lds_probe (built from tests/lds_probe.hip by the build
step) streams 16-byte LDS reads and writes from every CU."""
import os
import re
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import bench  # noqa: E402
from gpu_util import announce  # noqa: E402


@pytest.mark.gpu
def test_bench_lds_peaks_match_the_probe():
    exe = os.path.join(HERE, "lds_probe")
    if not os.path.exists(exe):
        raise RuntimeError(f"{exe} is missing: run __graft_entry__.build() first")
    announce("lds probe")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, check=True).stdout
    rate = {m.group(1): float(m.group(2))
            for m in re.finditer(r"^(\w+)\s+[\d.]+ ms\s+[\d.]+ TB/s\s+([\d.]+) B/clk/CU", out, re.M)}
    assert {"read_b128", "write_b128"} <= set(rate), out
    # the probe times at the nominal clock; the constants must be within 15 %
    assert abs(rate["read_b128"] / bench.LDS_READ_B_PER_CLK - 1) < 0.15, (rate, out)
    assert abs(rate["write_b128"] / bench.LDS_WRITE_B_PER_CLK - 1) < 0.15, (rate, out)
