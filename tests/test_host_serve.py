"""The render server's scheduler and the C entry points' host code, built with
AddressSanitizer and UndefinedBehaviorSanitizer against a fake HIP runtime (CPU only):
continuous batching, overflow retry, admission by the memory budget, waits racing with
statistics resets, latency from the arrival time, shutdown with queued requests, and the
stateless calls' argument handling (tests/host/serve_host_test.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_13339_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
ROCM_INCLUDE = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="needs g++ and the HIP runtime headers")
def test_server_and_entry_points_under_sanitizers(tmp_path):
    exe = str(tmp_path / "serve_host_test")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "veg_api.cpp"), os.path.join(CSRC, "veg_serve.cpp"),
           os.path.join(HOST, "fake_hip.cpp"), os.path.join(HOST, "serve_host_test.cpp"), "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all scenarios passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
