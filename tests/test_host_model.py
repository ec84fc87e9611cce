"""CPU: the driver's host-side pieces that touch no device
(paper_2504_18943_amd/csrc/ltlf_host.h) — the scheduler's region allocator
(first fit, top fit, placement at an offset, release with coalescing)
against a granule-by-granule model, and the workspace size model's
invariants (the carve-up fits, capacities grow with the workspace and stay
below the row limit, a smaller region's row store never starts after a
larger workspace's), and the search for a block that avoids given
intervals (which stages a job's stored levels when it takes the whole area)
against brute force.  Compiled with g++ from tests/host/host_check.cpp."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_allocator_and_size_model(tmp_path):
    exe = tmp_path / "host_check"
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-o", str(exe), os.path.join(HERE, "host", "host_check.cpp")],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
