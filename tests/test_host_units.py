"""Host-side units of the library, built with the system compiler against the
HIP headers and run on the CPU (tests/host_units.cpp):
  * the thread pool (packing, scattering, copy-out): short rounds issued back
    to back must each run every item exactly once with their own function. A
    worker waking late for a finished round once took an item of the next
    round with the old round's function (found under AddressSanitizer in the
    served workload);
  * the chunk schedule of staged transfers must tile every range exactly
    with non-empty chunks (its ramp once overflowed past 44 chunks)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1906_01128_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_pool_rounds_back_to_back(tmp_path):
    exe = tmp_path / "host_units"
    cmd = ["g++", "-std=c++17", "-O2", "-g", "-pthread", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(ROOT, "tests", "host_units.cpp"),
           os.path.join(CSRC, "dc_host.cpp"), "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe), "20000"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, f"pool stress failed ({r.returncode}): {r.stdout}{r.stderr[-2000:]}"
