"""Builds libdc.so (the HIP library behind include/dc.h) for gfx950 with hipcc.

Run `python -m paper_1906_01128_amd.build` (or __graft_entry__.build()).
Sources are compiled in parallel; the library is written next to this file
in _lib/ so that it travels with the source tree.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libdc.so")
SOURCES = ["dc_kernels.hip", "dc_scan.hip", "dc_host.cpp", "dc_plan.cpp", "dc_tree.cpp", "dc_chain.cpp", "dc_scalar.cpp", "dc_md.cpp", "dc_batch.cpp",
           "dc_server.cpp", "dc_noalloc.cpp"]
ARCH = os.environ.get("DC_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are disabled: plain scalar or float2 code only
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build_id():
    """Hash of the library sources: the autotuner keys its cached choices by it."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)) + ["../../include/dc.h"]:
        path = os.path.normpath(os.path.join(CSRC, name))
        if os.path.isfile(path):
            h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def _compile(src, obj, verbose, bid):
    cmd = [HIPCC, "-x", "hip", *FLAGS, f'-DDC_BUILD_ID="{bid}"', "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the GPU feature flag; that warning is harmless
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err and verbose:
        print(err, file=sys.stderr)
    return obj


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    objdir = os.path.join(OUT_DIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in srcs]
    bid = build_id()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose, bid), zip(srcs, objs)))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
