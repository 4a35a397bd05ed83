"""Host-only scheduler policy tests: builds tests/native/serve_core_test.cpp
with g++ (plain and ThreadSanitizer) and runs it.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "serve_core_test.cpp")


@pytest.mark.parametrize("san", ["", "thread"])
def test_scheduler_policy_with_mock_executor(tmp_path, san):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / f"serve_core_test{san}"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2602_15036_amd", "csrc"), SRC, "-o", str(exe)]
    if san:
        # GCC 11's TSan runtime misses the steady-clock condition wait; the
        # scheduler's system-clock wait path is used for this build.
        cmd[1:1] = [f"-fsanitize={san}", "-DLITHO_SERVE_SYSTEM_CLOCK_WAITS"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    if san:
        assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
