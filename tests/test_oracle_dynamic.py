"""Pins of the oracle's keyframe drop (sliding window, dynamic Hessian; in
the DSO integration of Sec. 4.2 every change of the keyframe set still cost
a new Hessian). GaussNewton.drop_frame(f) takes f's observations
out of the window and, mid-level, forms the IC system again from the rows of
J and the weights W0 kept at p(0). It is pinned to the level set-up of the
reduced problem (the observations removed from the input, the frame and the
points kept), which shares none of the drop's code path: the same reduced
system, the same steps."""
import numpy as np
import pytest

import scenes
from oracle.gn import GaussNewton, Problem

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def reduced_scene_arrays(sc, f):
    """Observation CSR of the scene without frame f's observations: those of
    points hosted by f and those with target f (points and frames kept)."""
    ptr, frames = [0], []
    for n in range(sc.n_points):
        obs = sc.obs_frame[sc.obs_ptr[n]:sc.obs_ptr[n + 1]]
        keep = [] if sc.host_frame[n] == f else [g for g in obs if g != f]
        frames.extend(keep)
        ptr.append(len(frames))
    return np.asarray(ptr, np.int64), np.asarray(frames, np.int64)


def reduced_problem(sc, f, poses, d):
    ptr, frames = reduced_scene_arrays(sc, f)
    return Problem(sc.images, sc.intrinsics, poses, sc.host_frame, sc.host_uv, d, ptr, frames, sc.pattern,
                   n_levels=sc.n_levels, huber_k=sc.huber_k)


@pytest.fixture(scope="module")
def mid_small():
    return scenes.mid(n_per_host=150)


@pytest.mark.parametrize("f", [6, 13])   # a host frame and a target-only frame
def test_ic_drop_equals_reduced_problem_setup(mid_small, f):
    """Dropped right after a level's start, the rebuilt IC system equals the
    reduced problem's set-up at the same p(0), and so do the next steps."""
    sc = mid_small
    a = GaussNewton(Problem.from_scene(sc), "ic")
    a.iterate(2, 2)             # move off the initial parameters first
    a.start_level(1)
    b = GaussNewton(reduced_problem(sc, f, a.poses, a.d), "ic")
    b.start_level(1)
    a.drop_frame(f)
    np.testing.assert_allclose(a.red.S, b.red.S, rtol=1e-12, atol=1e-12 * np.abs(b.red.S).max())
    np.testing.assert_allclose(a.red.Hdd, b.red.Hdd, rtol=1e-12)
    for _ in range(3):
        sa, sb = a.step(), b.step()
        assert sa["n_active"] == sb["n_active"]
        assert abs(sa["energy"] / sb["energy"] - 1) <= 1e-12
        assert abs(sa["max_disp_px"] - sb["max_disp_px"]) <= 1e-9
    np.testing.assert_allclose(a.poses, b.poses, rtol=0, atol=1e-12)
    np.testing.assert_allclose(a.d, b.d, rtol=1e-11)


def test_ic_drop_mid_level_keeps_p0(mid_small):
    """Dropped after iterations within a level, the system is the reduced
    problem's set-up at the level's p(0), not at the current parameters."""
    sc = mid_small
    a = GaussNewton(Problem.from_scene(sc), "ic")
    a.start_level(1)
    p0, d0 = a.poses.copy(), a.d.copy()
    a.step()
    a.step()
    a.drop_frame(6)
    b = GaussNewton(reduced_problem(sc, 6, p0, d0), "ic")
    b.start_level(1)
    np.testing.assert_allclose(a.red.S, b.red.S, rtol=1e-12, atol=1e-12 * np.abs(b.red.S).max())


def test_fc_drop_equals_reduced_problem(mid_small):
    sc = mid_small
    a = GaussNewton(Problem.from_scene(sc), "fc")
    a.iterate(1, 1)
    b = GaussNewton(reduced_problem(sc, 12, a.poses, a.d), "fc")
    b.start_level(1)
    a.drop_frame(12)
    for _ in range(2):
        sa, sb = a.step(), b.step()
        assert sa["n_active"] == sb["n_active"]
        assert abs(sa["energy"] / sb["energy"] - 1) <= 1e-12
    np.testing.assert_allclose(a.poses, b.poses, rtol=0, atol=1e-12)
    np.testing.assert_allclose(a.d, b.d, rtol=1e-11)


def test_dropped_frame_and_points_stay_put(mid_small):
    """The dropped frame's pose and the depths of the points it hosts no
    longer move (no observation constrains them), and the evaluation counts
    no residual of theirs."""
    sc = mid_small
    a = GaussNewton(Problem.from_scene(sc), "ic")
    a.start_level(0)
    a.drop_frame(6)
    hosted = sc.host_frame == 6
    pose6, dh = a.poses[6].copy(), a.d[hosted].copy()
    a.step()
    a.step()
    # a zero step recomposes the pose through p(0) (rounding only)
    np.testing.assert_allclose(a.poses[6], pose6, rtol=0, atol=1e-14)
    np.testing.assert_allclose(a.d[hosted], dh, rtol=1e-15)
    ev = a.evaluate(0)
    b = GaussNewton(reduced_problem(sc, 6, a.poses, a.d), "ic")
    assert ev["n_active"] == b.evaluate(0)["n_active"]


def test_gauge_frame_cannot_be_dropped(mid_small):
    a = GaussNewton(Problem.from_scene(mid_small), "ic")
    with pytest.raises(AssertionError):
        a.drop_frame(0)
