"""The server's host logic (queue, admission by footprint, arena, tickets,
poll/wait) under ThreadSanitizer and AddressSanitizer, on the CPU.

csrc/server.cpp is compiled with g++ against stand-ins for the HIP calls and
the solve entry points it uses (tests/host_server/mock_runtime.cpp); a
driver submits 900 requests from six threads and checks every result.  No
GPU code is built or run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2502_17963_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_server")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                                reason="needs g++ and the HIP headers")


@pytest.mark.parametrize("sanitizer", ["thread", "address"])
def test_server_host_logic_under_sanitizer(sanitizer, tmp_path):
    exe = str(tmp_path / f"stress_{sanitizer}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={sanitizer}", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + SRC,
           os.path.join(SRC, "server.cpp"), os.path.join(HERE, "mock_runtime.cpp"),
           os.path.join(HERE, "stress.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "done 900 bad 0" in out, out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out and "ERROR: AddressSanitizer" not in out
