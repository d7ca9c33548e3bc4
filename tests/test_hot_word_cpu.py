"""The FP32 hot word's candidacy encoding, checked on the host.

tests/hot_word_check.cpp includes the kernels' own device.h and checks, for
epochs and next-pass steps across the offset's range, that cell, class and
candidacy survive encoding, that hw_due fires exactly at the first pass with
knext <= k (the oracle's candidacy rule, oracle/sim.py), that a sort's
re-expression keeps the candidacy, and that hw_move changes the cell only.
It is built with hipcc for the host (no GPU needed).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2308_13092_amd", "csrc")


def test_hot_word_encoding(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "hot_word_check"
    subprocess.run([hipcc, "-std=c++17", "-O2", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-I", CSRC, os.path.join(HERE, "hot_word_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
