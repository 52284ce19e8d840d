"""Host-side contract of bench.py (no GPU): the one-GPU guard, and measured L2-miss
traffic reported only for the kernel sources the counters were taken on."""
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


def test_measured_traffic_follows_the_kernel_sources(monkeypatch):
    import bench
    h = hashlib.sha256()
    for f in ("pba_kernels.hip", "pba_solver.hip", "pba_depth.hpp", "pba_device.hpp", "pba_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1704_06967_amd", "csrc", f), "rb").read())
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "sources_sha256_16", h.hexdigest()[:16])
    assert bench.measured_traffic("k_ic_residual", "mid") == bench.MEASURED_TRAFFIC["k_ic_residual"]["mid"]
    assert bench.measured_traffic("k_ic_residual", "precision") == bench.MEASURED_TRAFFIC["k_ic_residual"]["precision"]
    assert bench.measured_traffic("k_ic_step", "mid") == bench.MEASURED_TRAFFIC["k_ic_step"]["mid"]
    assert bench.measured_traffic("k_ic_step", "precision") is None   # not measured
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "sources_sha256_16", "0" * 16)
    assert bench.measured_traffic("k_ic_residual", "mid") is None
    assert bench.measured_traffic("k_ic_step", "mid") is None
    # the joint linearization has a table of its own, keyed on its own sources
    h = hashlib.sha256()
    for f in ("pba_affine.hip", "pba_affine.hpp", "pba_device.hpp", "pba_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1704_06967_amd", "csrc", f), "rb").read())
    monkeypatch.setitem(bench.MEASURED_TRAFFIC_AFFINE, "sources_sha256_16", h.hexdigest()[:16])
    assert bench.measured_traffic("k_aff_linearize", "mid") == bench.MEASURED_TRAFFIC_AFFINE["k_aff_linearize"]["mid"]
    assert bench.measured_traffic("k_aff_linearize", "precision") is None
    monkeypatch.setitem(bench.MEASURED_TRAFFIC_AFFINE, "sources_sha256_16", "0" * 16)
    assert bench.measured_traffic("k_aff_linearize", "mid") is None



def test_module_level_helpers_are_defined():
    import bench
    for name in ("METRIC", "log", "level_pixels", "_pairs", "_unique_texels", "frontend_section",
                 "_predicted_positions", "roofline_obj", "measured_traffic"):
        assert hasattr(bench, name), name
