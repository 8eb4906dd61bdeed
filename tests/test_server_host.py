"""The server's host logic (queue, admission by footprint, arena, tickets,
poll/wait) under ThreadSanitizer, AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

Two harnesses, both compiled with g++ against stand-ins for the HIP runtime
(no GPU code is built or run):
  * stress.cpp + mock_runtime.cpp: csrc/server.cpp alone, with the solve
    entry points stubbed; six threads submit 900 requests;
  * serving_stress.cpp + mock_hip.cpp + mock_kernels.cpp: the real server,
    C ABI and solve driver (triple tables, workspace layout, explicitly built
    graphs, events, two-stream pipeline) on an emulated runtime whose
    kernels check every device range they touch.  Modes: six client threads;
    the serving stream's own 256 fragment shapes with a submitter that
    allocates, fills, submits, polls, frees and empties its allocator cache
    concurrently with the server's slots; several threads consuming one
    ticket and a destroy while waiters are blocked.
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

FLAGS = {"thread": ["-fsanitize=thread"],
         "address": ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]}
ENV = {"TSAN_OPTIONS": "halt_on_error=1", "ASAN_OPTIONS": "halt_on_error=1:detect_leaks=0",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _compile(sources, exe, sanitizer):
    cmd = ["g++", "-std=c++17", "-O1", "-g", *FLAGS[sanitizer], "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + SRC, *sources, "-o", exe,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]


def _run(cmd, timeout=900):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=dict(os.environ, **ENV))
    out = r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out and "MOCK-HIP FAULT" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


@pytest.mark.parametrize("sanitizer", ["thread", "address"])
def test_server_host_logic_under_sanitizer(sanitizer, tmp_path):
    exe = str(tmp_path / f"stress_{sanitizer}")
    _compile([os.path.join(SRC, "server.cpp"), os.path.join(HERE, "mock_runtime.cpp"),
              os.path.join(HERE, "stress.cpp")], exe, sanitizer)
    assert "done 900 bad 0" in _run([exe])


@pytest.fixture(scope="module", params=["address", "thread"])
def serving_exe(request, tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("serving") / f"serving_stress_{request.param}")
    _compile(["-x", "c++", os.path.join(SRC, "solve.hip"), os.path.join(SRC, "batch.hip"), "-x", "none",
              os.path.join(SRC, "server.cpp"),
              os.path.join(SRC, "abi.cpp"), os.path.join(SRC, "sizes.cpp"), os.path.join(HERE, "mock_hip.cpp"),
              os.path.join(HERE, "mock_kernels.cpp"), os.path.join(HERE, "serving_stress.cpp")], exe,
             request.param)
    return request.param, exe


def test_serving_client_threads(serving_exe):
    _, exe = serving_exe
    assert "threads: done 360 bad 0" in _run([exe, "threads"])


def test_serving_shared_ticket_and_destroy_with_waiters(serving_exe):
    """Two or three threads consume one ticket (exactly one gets the result,
    the others BQC_ENOTFOUND, and no waiter reads a freed request); then the
    server is destroyed while twelve waiters are blocked inside bqc_t_wait."""
    _, exe = serving_exe
    assert "consumers: bad 0" in _run([exe, "consumers"])


def test_serving_stream_shapes(serving_exe, tmp_path):
    """The serving stream's fragment shapes (nocc 8..40, nvir up to 400; real
    triple tables, batch sizes and graphs of up to 64 batches) with the
    benchmark's submit / poll / free / empty-cache pattern, graphs and direct
    launches (ThreadSanitizer: the first 128 fragments)."""
    from synth import serving_stream
    san, exe = serving_exe
    shapes = tmp_path / "shapes.txt"
    shapes.write_text("".join(f"{s['nocc']} {s['nvir']}\n" for s in serving_stream(256)))
    n = 256 if san == "address" else 128
    for direct in ("0", "1"):
        out = _run([exe, "stream", str(shapes), direct, str(n)])
        assert f"stream: done {n} bad 0" in out, out[-2000:]


def test_serving_failure_isolation(serving_exe):
    """Requests made to fail at admission (BQC_ENOMEM) or after their solve
    (BQC_EDEVICE) by injection, and requests cancelled while queued
    (BQC_ECANCELED), among 90 requests on three slots: every other request's
    energy is unchanged, every ticket is consumed once, graphs and direct
    launches."""
    _, exe = serving_exe
    for direct in ("0", "1"):
        out = _run([exe, "faults", direct])
        assert "bad 0" in out and "faults: ok" in out, out[-2000:]


def test_batch_driver(serving_exe):
    """bqc_t_energy_batch's host driver (batch plan, tables, grouped-launch
    entries of every round) on the stand-in runtime: fragments of mixed
    sizes in several rounds, host and device inputs, every energy equal to
    the fragment's solve alone."""
    _, exe = serving_exe
    assert "batch: bad 0" in _run([exe, "batch"])
