"""The C ABI without a GPU: exported symbols, struct layout, defaults, argument
validation (which runs before any device work) and status strings."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pba.h")

pba = pytest.importorskip("paper_1704_06967_amd.pba")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pba_[a-z_]+)\s*\(", txt)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert len(names) >= 14
    lib = C.CDLL(pba.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(pba.EXPORTED) == names


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    fields = {
        "pba_config": [f for f, _ in pba.pba_config._fields_],
        "pba_iter_stats": [f for f, _ in pba.pba_iter_stats._fields_],
        "pba_result": [f for f, _ in pba.pba_result._fields_],
        "pba_timing": [f for f, _ in pba.pba_timing._fields_],
        "pba_tune_report": [f for f, _ in pba.pba_tune_report._fields_],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for s, fs in fields.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for s, fs in fields.items():
        cls = getattr(pba, s)
        assert int(got[s]) == C.sizeof(cls), s
        for f in fs:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, f"{s}.{f}"


def test_config_default_values():
    cfg = pba.default_config()
    assert cfg.mode == pba.PBA_IC_PROXY and cfg.precision == pba.PBA_FP32
    assert cfg.n_levels == 1 and cfg.pattern_n == 8
    assert abs(cfg.huber_k - 9 / 255) < 1e-15 and cfg.damping_rel == 1e-6
    assert cfg.pinned_frame == 0 and cfg.n_windows == 1 and cfg.stream is None
    pat = np.array(cfg.pattern_uv[:16]).reshape(8, 2)
    import scenes

    assert np.array_equal(pat, scenes.PATTERN8)


@pytest.mark.parametrize("field,value,msg", [
    ("mode", 7, "mode"), ("precision", 9, "precision"), ("n_levels", 0, "n_levels"),
    ("n_levels", 5, "n_levels"), ("pattern_n", 0, "pattern_n"), ("pattern_n", 9, "pattern_n"),
    ("huber_k", 0.0, "huber_k"), ("huber_k", float("nan"), "huber_k"), ("damping_rel", -1.0, "damping_rel"),
    ("damping_rel", float("inf"), "damping_rel"), ("pinned_frame", -2, "pinned_frame"), ("solver", 3, "solver"),
    ("n_windows", 0, "n_windows"), ("n_windows", 5000, "n_windows"), ("flags", 8, "flag"),
])
def test_create_rejects_invalid_config(field, value, msg):
    cfg = pba.default_config()
    setattr(cfg, field, value)
    h = C.c_void_p()
    s = pba.pba_create(C.byref(cfg), C.byref(h))
    assert s == pba.PBA_E_INVALID
    assert msg in pba.last_error()
    assert not h.value


def test_create_rejects_large_pattern_offsets():
    cfg = pba.default_config()
    cfg.pattern_uv[3] = 5
    h = C.c_void_p()
    assert pba.pba_create(C.byref(cfg), C.byref(h)) == pba.PBA_E_INVALID


def test_null_arguments():
    assert pba.pba_create(None, None) == pba.PBA_E_INVALID
    assert pba.pba_config_default(None) == pba.PBA_E_INVALID
    assert pba.pba_iterate(None, 0, 1, None) == pba.PBA_E_INVALID
    assert pba.pba_set_frames(None, 0, 1, 8, 8, None, None, None, 0) == pba.PBA_E_INVALID
    assert pba.pba_evaluate(None, 0, None) == pba.PBA_E_INVALID
    assert pba.pba_set_affine(None, None) == pba.PBA_E_INVALID
    assert pba.pba_get_affine(None, None) == pba.PBA_E_INVALID
    pba.pba_destroy(None)


def test_status_strings():
    for k in ("PBA_OK", "PBA_E_INVALID", "PBA_E_STATE", "PBA_E_OOM", "PBA_E_DEVICE", "PBA_E_NUMERIC",
              "PBA_E_NOT_CONVERGED"):
        assert pba.status_string(getattr(pba, k)) == k


def test_valid_config_without_gpu_reports_device_error():
    if os.path.exists("/dev/kfd"):
        pytest.skip("a GPU is present")
    cfg = pba.default_config()
    h = C.c_void_p()
    assert pba.pba_create(C.byref(cfg), C.byref(h)) == pba.PBA_E_DEVICE


def header_define(name):
    m = re.search(rf"#define\s+{name}\s+(\d+)", open(HEADER).read())
    return int(m.group(1))


@pytest.mark.parametrize("field,value", [
    ("n_windows", 1), ("n_windows", 2), ("n_windows", None), ("flags", 1), ("flags", 2), ("flags", 3),
    ("n_levels", 4), ("pattern_n", 1), ("pinned_frame", -1), ("huber_k", float("inf")), ("damping_rel", 0.0),
])
def test_create_accepts_documented_limits(field, value):
    """Every value the header documents as valid passes validation (without a GPU
    the call then fails only for the missing device); one past the documented
    window limit does not."""
    if os.path.exists("/dev/kfd"):
        pytest.skip("a GPU is present")
    assert header_define("PBA_MAX_WINDOWS") == pba.PBA_MAX_WINDOWS
    assert header_define("PBA_FE_MAX_CELLS") == pba.PBA_FE_MAX_CELLS
    assert header_define("PBA_FE_MAX_RADIUS") == pba.PBA_FE_MAX_RADIUS
    cfg = pba.default_config()
    setattr(cfg, field, pba.PBA_MAX_WINDOWS if value is None else value)
    h = C.c_void_p()
    assert pba.pba_create(C.byref(cfg), C.byref(h)) == pba.PBA_E_DEVICE, pba.last_error()
    cfg.n_windows = pba.PBA_MAX_WINDOWS + 1
    assert pba.pba_create(C.byref(cfg), C.byref(h)) == pba.PBA_E_INVALID


def test_noalloc_solve_rejects_sizes_before_device_work():
    """pba_solve_dense_noalloc validates n and its pointers before any HIP call
    (no GPU here): sizes outside 1..PBA_NOALLOC_MAX_N and NULL buffers."""
    import ctypes as C
    for n in (0, -3, pba.PBA_NOALLOC_MAX_N + 1):
        assert pba.pba_solve_dense_noalloc(n, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None, None) == pba.PBA_E_INVALID
        assert "768" in pba.last_error()
    assert pba.pba_solve_dense_noalloc(16, None, C.c_void_p(8), C.c_void_p(8), None, None) == pba.PBA_E_INVALID

