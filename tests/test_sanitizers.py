"""The host library and the CPU oracle under sanitizers, on the CPU.

tests/sanitize/host_checks.cpp drives the planner against the oracle, the deep
copy and copy back through the pinned staging ring, the batched form's shape
checks and autotuner, and the served form from several submitting threads; tests/sanitize/mock_hip.cpp stands in for the HIP
runtime (host memory as device memory, one worker thread per stream, so
copies and event records really run asynchronously to their callers).

  * AddressSanitizer + UndefinedBehaviorSanitizer (g++): every mode.
  * ThreadSanitizer (the ROCm LLVM clang++, whose runtime intercepts
    pthread_cond_clockwait; GCC 11's does not, and then reports every timed
    condition-variable wait as a double lock): the deep copy's ring and pool
    threads and the server's submit, issue, completion and wait threads.

Host code only: no GPU code is built with a sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_01128_amd", "csrc")
HOST_SOURCES = ["dc_host", "dc_plan", "dc_tree", "dc_server", "dc_chain", "dc_scalar", "dc_md", "dc_batch"]
LLVM = "/opt/rocm/llvm/bin"


def _build(out, cc, cxx, san):
    os.makedirs(out, exist_ok=True)
    inc = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-I", os.path.join(ROOT, "fixtures"), "-I", os.path.join(ROOT, "oracle")]
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", *san]
    objs = []
    for src in ("fixtures/fx.c", "oracle/oracle.c"):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        r = subprocess.run([cc, "-std=c11", *flags, "-c", os.path.join(ROOT, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    srcs = [os.path.join(ROOT, "tests", "sanitize", f) for f in ("host_checks.cpp", "mock_hip.cpp")]
    srcs += [os.path.join(CSRC, f + ".cpp") for f in HOST_SOURCES]
    exe = os.path.join(out, "host_checks")
    r = subprocess.run([cxx, "-std=c++17", *flags, "-pthread", *inc, *srcs, *objs, "-lm", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, modes, env):
    r = subprocess.run([exe, *modes], capture_output=True, text=True, timeout=600, env={**os.environ, **env},
                       cwd=ROOT)
    report = r.stdout[-2000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer", "ERROR: LeakSanitizer"):
        assert marker not in r.stderr, report
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_address_and_undefined_behaviour(tmp_path):
    exe = _build(str(tmp_path / "asan"), "gcc", "g++",
                 ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    out = _run(exe, ["plan", "copy", "batch", "server"], {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                                                           "UBSAN_OPTIONS": "print_stacktrace=1"})
    for mode in ("plan", "copy", "batch", "server"):
        assert f"{mode}: 0 failures" in out, out


@pytest.mark.skipif(not os.path.exists(os.path.join(LLVM, "clang++")) or not os.path.isdir("/opt/rocm/include"),
                    reason="needs the ROCm LLVM clang++ and the ROCm headers")
def test_threads(tmp_path):
    exe = _build(str(tmp_path / "tsan"), os.path.join(LLVM, "clang"), os.path.join(LLVM, "clang++"),
                 ["-fsanitize=thread"])
    out = _run(exe, ["copy", "batch", "server"], {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})
    for mode in ("copy", "batch", "server"):
        assert f"{mode}: 0 failures" in out, out
