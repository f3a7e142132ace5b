"""The host driver and the solve server (planner, batched factor/apply/solve,
admission, LRU eviction, batching) built for the CPU against a stand-in HIP
runtime (tests/host_stub: zeroed host memory, no-op kernel launches) and run
under AddressSanitizer.  Checks the host logic only: memory errors, request
accounting, evictions under a small budget; the numerics are covered by the
GPU tests."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STUB = os.path.join(ROOT, "tests", "host_stub")
CSRC = os.path.join(ROOT, "paper_2310_15458_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_logic_under_asan(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address",
           "-I", STUB, "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           "-x", "c++", os.path.join(CSRC, "rss_host.cpp"),
           "-x", "c++", os.path.join(CSRC, "rss_server.cpp"),
           os.path.join(STUB, "launch_stubs.cpp"), os.path.join(STUB, "driver.cpp"),
           "-o", exe, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout[-2000:])
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "OK" in run.stdout
