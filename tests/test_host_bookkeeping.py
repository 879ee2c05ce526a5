"""Host-side bookkeeping of the request server (stripe index and store ring),
checked on the CPU: a small C++ driver built with the host compiler runs
randomised operations against std::unordered_map and a brute-force overlap
check (tests/host/stripe_index_check.cpp)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_stripe_index_and_ring(tmp_path):
    exe = tmp_path / "stripe_index_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    os.path.join(HERE, "host", "stripe_index_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
