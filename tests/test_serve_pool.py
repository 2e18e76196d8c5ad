"""Admission by device bytes in the query server, on the host with a fake
budget: the batch layout, the first-fit pool and the batch-formation rule
of paper_1910_02611_amd/csrc/serve_pool.hpp (the code the server runs),
driven by tests/csrc/serve_pool_test.cpp (g++, no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_pool_admission_on_host(tmp_path):
    exe = str(tmp_path / "serve_pool_test")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-fsanitize=address,undefined",
           "-I", os.path.join(ROOT, "paper_1910_02611_amd", "csrc"), "-o", exe,
           os.path.join(ROOT, "tests", "csrc", "serve_pool_test.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "serve pool ok" in r.stdout
