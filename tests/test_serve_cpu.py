"""The serving scheduler core on the CPU, driven by a fake executor (no GPU):
budget and slot admission, FIFO order, continuous batching, failure
propagation, timeouts, shutdown, percentile arithmetic. Built twice with g++:
plain and with ThreadSanitizer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "serve_core_test.cpp")
INC = os.path.join(ROOT, "paper_2406_09266_amd", "csrc")


@pytest.mark.parametrize("sanitize", [None, "thread"])
def test_serve_core(tmp_path, sanitize):
    exe = tmp_path / "serve_core_test"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread", "-I", INC, SRC, "-o", str(exe)]
    if sanitize:
        cmd.insert(1, f"-fsanitize={sanitize}")
    subprocess.check_call(cmd)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL PASS" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
