"""Host layout conversion of the C ABI (hl_init / hl_export), compiled from
paper_1808_10481_amd/csrc/hl_host_layout.hpp with g++ under AddressSanitizer
and UBSan and run on the CPU (tests/host_layout_check.cpp)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_layout_round_trip_under_sanitizers(tmp_path):
    exe = tmp_path / "host_layout_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-pthread", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1808_10481_amd", "csrc"),
           os.path.join(HERE, "host_layout_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])
