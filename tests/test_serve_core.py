"""The serving scheduler's policy (ServeCore) against a mock executor, on the
CPU: serve_core_test.cpp is built with g++ from the library's own
serve_core.cpp, once plainly and once with ThreadSanitizer, and run.  It covers
admission by HBM budget, strict FIFO order, slot limits, VP_ECAPACITY, ticket
release, the VP_EBUSY protocol, eviction, a per-job admission failure, a
device failure that ends every running job, draining and a multi-threaded
stress run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2005_09316_amd", "csrc")


@pytest.mark.parametrize("sanitizer", [None, "thread"])
def test_serve_core_mock_executor(tmp_path, sanitizer):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "serve_core_test")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread", "-Wall",
           "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "serve_core_test.cpp"), os.path.join(CSRC, "serve_core.cpp"),
           "-o", exe]
    if sanitizer:
        cmd.insert(1, "-fsanitize=" + sanitizer)
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr, r.stderr
    assert r.stdout.count("PASS") == 10 and "FAIL" not in r.stdout, r.stdout
