"""GPU parity of reduced pose systems larger than one workgroup's LDS (6F > 180):
the tiled Cholesky (FP64 MFMA tile products), its tile-blocked triangular solves
and the IC inverse built from it, against the FP64 oracle.

The scene is the mid ellipsoid orbit with 40 frames (6F = 240: seven full 32 x 32
tiles and a ragged 16-row tail), 5 hosts x 1000 points.
"""
import numpy as np
import pytest

import scenes
from oracle.gn import GaussNewton, Problem
from tests.oracle_refs import depth_errors_ok, rot_err, trans_rel_err

pytestmark = pytest.mark.gpu

pba = pytest.importorskip("paper_1704_06967_amd.pba")


def make(scene, mode, precision, **kw):
    s = pba.Solver(mode=pba.PBA_IC_PROXY if mode == "ic" else pba.PBA_FC, precision=precision,
                   n_levels=scene.n_levels, pattern=scene.pattern, huber_k=scene.huber_k, **kw)
    s.set_scene(scene)
    return s


@pytest.fixture(scope="module")
def mid40():
    sc = scenes.mid(n_per_host=1000, n_frames=40)
    assert 6 * sc.n_frames > 180
    return sc


@pytest.mark.parametrize("mode", ["fc", "ic"])
def test_tiled_first_step_fp64(mid40, mode):
    """S, b and the step of the first level-0 iteration."""
    s = make(mid40, mode, 0)
    s.iterate(0, 1)
    gn = GaussNewton(Problem.from_scene(mid40), mode)
    gn.iterate(0, 1)
    S = s.fetch(pba.PBA_DBG_S)
    Sref = gn.last["S"]
    np.testing.assert_allclose(S, Sref, rtol=1e-10, atol=1e-10 * np.abs(Sref).max())
    b = s.fetch(pba.PBA_DBG_B)
    np.testing.assert_allclose(b, gn.last["b"], rtol=1e-9, atol=1e-11 * np.abs(gn.last["b"]).max())
    dth = s.fetch(pba.PBA_DBG_DTHETA)
    ref = -np.linalg.solve(Sref, gn.last["b"])
    # normwise: S has a condition number of ~2e7 here, so two backward-stable
    # solves agree to about cond x eps relative to the solution's norm
    assert np.linalg.norm(dth - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("mode", ["fc", "ic"])
def test_tiled_iterations_fp64(mid40, mode):
    s = make(mid40, mode, 0)
    gn = GaussNewton(Problem.from_scene(mid40), mode)
    for level in (2, 1, 0):
        st = s.iterate(level, 3)
        ost = gn.iterate(level, 3)
        for a, o in zip(st, ost):
            assert a["n_active"] == o["n_active"]
            assert abs(a["energy"] / o["energy"] - 1) <= 1e-9
    poses, d = s.get_params()
    # FP64 on both sides: agreement to rounding amplified by cond(S) ~ 1e7
    assert rot_err(poses, gn.poses).max() <= 1e-8
    assert trans_rel_err(poses, gn.poses).max() <= 1e-8
    assert np.abs(d / gn.d - 1).max() <= 1e-8


@pytest.mark.parametrize("mode", ["fc", "ic"])
def test_tiled_iterations_fp32(mid40, mode):
    s = make(mid40, mode, 1)
    gn = GaussNewton(Problem.from_scene(mid40), mode)
    for level in (2, 1, 0):
        s.iterate(level, 8)
        gn.iterate(level, 8)
    poses, d = s.get_params()
    assert rot_err(poses, gn.poses).max() <= 1e-5
    assert trans_rel_err(poses, gn.poses).max() <= 1e-5
    ok, q99, worst = depth_errors_ok(d, gn.d)
    assert ok, (q99, worst)
    ev, oev = s.evaluate(0), gn.evaluate(0)
    assert abs(ev["rmse"] / oev["rmse"] - 1) <= 1e-4


def test_ic_split_solve_iterations_fp64():
    """IC with 6F = 288 > 256 unknowns on one window: the step's product with
    S^{-1} runs between the two stages of the solve (many workgroups), and the
    window's poses, pair geometry and index lists fit the solve's LDS cache, so
    the second stage reads dtheta from there."""
    sc = scenes.mid(n_per_host=400, n_frames=48)
    s = make(sc, "ic", 0)
    gn = GaussNewton(Problem.from_scene(sc), "ic")
    for level in (2, 1, 0):
        st = s.iterate(level, 3)
        ost = gn.iterate(level, 3)
        for a, o in zip(st, ost):
            assert a["n_active"] == o["n_active"]
            assert abs(a["energy"] / o["energy"] - 1) <= 1e-9
    poses, d = s.get_params()
    assert rot_err(poses, gn.poses).max() <= 1e-8
    assert trans_rel_err(poses, gn.poses).max() <= 1e-8
    assert np.abs(d / gn.d - 1).max() <= 1e-8


def test_ic_many_points_separate_kernels_fp64():
    """IC on one window with more points (36 000) than one round of the fused
    solve + depth-step grid covers: the solve and the depth step run as
    separate kernels. Level 2, three iterations against the oracle."""
    sc = scenes.mid(n_per_host=7200)
    s = make(sc, "ic", 0)
    gn = GaussNewton(Problem.from_scene(sc), "ic")
    st = s.iterate(2, 3)
    ost = gn.iterate(2, 3)
    for a, o in zip(st, ost):
        assert a["n_active"] == o["n_active"]
        assert abs(a["energy"] / o["energy"] - 1) <= 1e-9
    poses, d = s.get_params()
    assert rot_err(poses, gn.poses).max() <= 1e-8
    assert trans_rel_err(poses, gn.poses).max() <= 1e-8
    assert np.abs(d / gn.d - 1).max() <= 1e-8
