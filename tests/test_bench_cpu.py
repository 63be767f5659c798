"""The parts of bench.py's output contract that need no GPU: the refusal of
more than one GPU, the HBM-traffic lookup (reported only while the kernel
source is the one the counters were taken with), and the CPU baseline's
fields."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert r.stdout == ""
    assert "one GPU" in r.stderr


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "paper_1906_01128_amd" / "csrc"
    src.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (src / "dc_kernels.hip").write_bytes(b"kernels, version 1\n")
    sha = hashlib.sha256(b"kernels, version 1\n").hexdigest()
    (tmp_path / "profiles" / "hbm_counters.txt").write_text(
        "# workload kernel kernels_sha256 fetch_kib write_kib traffic_bytes\n"
        f"linear k_stream_deref {sha} 65569.0 131072.0 268503040\n"
        f"batched k_leaf_tiles {'0' * 64} 1.0 1.0 4096\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic("linear", "k_stream_deref") == 268503040
    assert bench.traffic("linear", "k_stream_resolved") is None    # no entry
    assert bench.traffic("batched", "k_leaf_tiles") is None        # taken with another source
    (src / "dc_kernels.hip").write_bytes(b"kernels, version 2\n")
    assert bench.traffic("linear", "k_stream_deref") is None       # the source changed since
    os.remove(tmp_path / "profiles" / "hbm_counters.txt")
    assert bench.traffic("linear", "k_stream_deref") is None


def test_cpu_baseline_fields():
    import bench
    b = bench.cpu_baseline_linear(None, passes=1)
    assert b["kind"] == "oracle" and b["cores"] == 1 and b["unit"] == "GB/s"
    assert b["value"] > 0 and b["seconds"] > 0
    assert "1 fma passes x 2 modes" in b["sample"]


def test_cpu_baseline_md_fields():
    """The batched workload's baseline: one thread on a sample, then every
    simulation over the CPUs available, each credited with the GPU step's
    algorithmic bytes of the same simulations."""
    import bench
    import fixtures as fx
    t = fx.md(nsims=40)
    b = bench.cpu_baseline_md(t, nsample=10, max_threads=4)
    assert b["kind"] == "oracle" and b["unit"] == "GB/s" and b["value"] > 0
    assert 1 <= b["cores"] <= 4 and b["cores"] <= b["cpus_available"]
    assert b["cpu_model"] and "all 40 simulations" in b["sample"]
    st = b["single_thread"]
    assert st["cores"] == 1 and st["value"] > 0 and "first 10 simulations" in st["sample"]
    # the credited bytes are those the GPU step moves for the same simulations
    from paper_1906_01128_amd import dc
    p = dc.Plan(dc.Schema(t.types), t.root_type, t.roots[:10])
    assert st["bytes"] == bench.md_step_bytes(p.info())
    i = p.info()
    assert st["bytes"] == 2 * i.leaf_bytes + 2 * (16 * i.nslots_nonnull + 8 * i.nslots + 16 * i.nobjects)
