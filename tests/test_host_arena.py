"""Host logic on the CPU: the serving loop's output arena (zg_arena.h),
compiled on its own with g++ and checked against a byte-map model."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2405_19493_amd", "csrc")


def test_arena_against_model(tmp_path):
    exe = str(tmp_path / "arena_check")
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", CSRC,
                        os.path.join(HERE, "host", "arena_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stdout + r.stderr)
    out = subprocess.run([exe, "20000"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
