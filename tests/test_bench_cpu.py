"""Host-side contract of bench.py (no GPU): the one-GPU guard, and measured HBM
traffic reported only for the kernel source the counters were taken on."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""   # no result line


def test_measured_traffic_follows_the_kernel_source(monkeypatch):
    import bench
    src = os.path.join(ROOT, "paper_1704_06967_amd", "csrc", "pba_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "kernels_sha256_16", sha)
    assert bench.measured_traffic("mid") == bench.MEASURED_TRAFFIC["mid"]
    assert bench.measured_traffic("precision") == bench.MEASURED_TRAFFIC["precision"]
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "kernels_sha256_16", "0" * 16)
    assert bench.measured_traffic("mid") is None
