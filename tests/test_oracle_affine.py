"""Pins of the affine-brightness oracle (oracle/affine.py) against exact
zero residuals, finite differences and the paper's residual at a = b = 0."""
import numpy as np
import pytest

import scenes
from oracle import affine as AF
from oracle import geometry as G
from oracle import residuals as RS
from oracle import solver as SV
from oracle.gn import Problem
from scenes.brightness import brighten, seeded_ab
from scenes.planar import planar


def _problem(sc, images, poses=None, d=None):
    return Problem(images, sc.intrinsics, sc.poses_init if poses is None else poses, sc.host_frame, sc.host_uv,
                   sc.inv_depth_init if d is None else d, sc.obs_ptr, sc.obs_frame, sc.pattern,
                   n_levels=sc.n_levels, huber_k=sc.huber_k)


@pytest.mark.parametrize("levels", [1, 2])
def test_brightened_planar_residuals_vanish_at_the_truth(levels):
    # the planar images are affine in their pixels, so are their brightened
    # versions, and bilinear sampling is exact: r == 0 at the true parameters,
    # which fixes the gain's direction (e^{a_h - a_f}) and both offsets' sides
    sc = planar(n_levels=levels, n_frames=4)
    ab = seeded_ab(sc.n_frames, 3)
    P = _problem(sc, brighten(sc.images, ab), sc.poses_gt, sc.inv_depth_gt)
    for level in range(levels):
        r, valid, _, _, _ = AF.affine_residuals(P, P.layout(level), sc.poses_gt, sc.inv_depth_gt, ab)
        assert valid.mean() > 0.8 and np.abs(r[valid]).max() < 1e-6
    # the wrong direction of the gain leaves residuals of the brightness change's size
    r, _, _, _, _ = AF.affine_residuals(P, P.layout(0), sc.poses_gt, sc.inv_depth_gt, -ab)
    assert np.abs(r[valid]).max() > 1e-2


def test_zero_brightness_is_the_papers_residual():
    sc = scenes.tiny()
    P = _problem(sc, sc.images)
    L = P.layout(0)
    r, valid, _, _, g = AF.affine_residuals(P, L, sc.poses_init, sc.inv_depth_init, np.zeros((sc.n_frames, 2)))
    r0, valid0, _, _ = RS.warp_residuals(P, L, sc.poses_init, sc.inv_depth_init)
    assert np.array_equal(valid, valid0) and np.array_equal(r, r0) and (g == 1.0).all()


def _fd_check(sc, images, ab0, cols, rtol):
    P = _problem(sc, images)
    L = P.layout(0)
    r, valid, q, If, g = AF.affine_residuals(P, L, sc.poses_init, sc.inv_depth_init, ab0)
    Jg, Jp = AF.affine_jacobian(P, L, sc.poses_init, sc.inv_depth_init, ab0, q, If, g)
    A, B = SV.pair_maps(L, sc.poses_init)
    J = AF.absolute_jacobian(L, Jg, Jp, A, B, sc.n_frames, sc.n_points).toarray()
    F6 = 6 * sc.n_frames
    h = 1e-6
    R, t = G.unpack(sc.poses_init)
    for c in cols:
        vals = []
        for s in (1.0, -1.0):
            dp = np.zeros(F6)
            dab = np.zeros((sc.n_frames, 2))
            dd = np.zeros(sc.n_points)
            if c < F6:
                dp[c] = s * h
            elif c < 8 * sc.n_frames:
                dab.reshape(-1)[c - F6] = s * h
            else:
                dd[c - 8 * sc.n_frames] = s * h
            d6 = dp.reshape(-1, 6)
            Rn, tn = G.boxplus_pose(R, t, d6[:, :3], d6[:, 3:])
            rr, _, _, _, _ = AF.affine_residuals(P, L, G.pack(Rn, tn), sc.inv_depth_init + dd, ab0 + dab)
            vals.append(rr)
        fd = (vals[0] - vals[1]) / (2 * h)
        m = valid
        assert np.allclose(J[m, c], fd[m], rtol=rtol, atol=rtol * np.abs(fd[m]).max() + 1e-9), c


def test_brightness_columns_match_finite_differences():
    # the brightness columns are analytic in (a, b): exact on any image
    sc = scenes.tiny()
    ab = seeded_ab(sc.n_frames, 4)
    ab0 = ab + np.array([[0.0, 0.0]] + [[0.02, -0.01]] * (sc.n_frames - 1))
    _fd_check(sc, brighten(sc.images, ab), ab0, [6 * sc.n_frames + k for k in range(2 * sc.n_frames)], 1e-6)


def test_geometry_columns_carry_the_gain():
    # on the planar problem the central-difference gradient is the bilinear
    # image's exact derivative, so the FC Jacobian scaled by the gain matches
    # finite differences of the brightened residual in every column
    sc = planar(n_levels=1, n_frames=3)
    ab = seeded_ab(sc.n_frames, 7)
    F = sc.n_frames
    cols = list(range(6, 6 * F)) + [6 * F + k for k in range(2, 2 * F)] + [8 * F + k for k in range(0, sc.n_points, 7)]
    # (float32 images: the interpolant is affine to their rounding, ~1e-5 relative)
    _fd_check(sc, brighten(sc.images, ab), ab * 0.5, cols, 1e-4)


def test_planar_brightness_change_is_recovered_to_zero_residual():
    sc = planar(n_levels=1, n_frames=4)
    ab = seeded_ab(sc.n_frames, 5)
    P = _problem(sc, brighten(sc.images, ab), sc.poses_gt, sc.inv_depth_gt)
    gn = AF.AffineFC(P)            # starts from a = b = 0 at the true geometry
    first = gn.iterate(0, 1)[0]
    assert first["rmse"] > 1e-3
    gn.iterate(0, 12)
    # down to the float32 rounding of the images (~6e-8 at 0.5)
    assert gn.history[-1]["rmse"] < 1e-6
    r, valid, _, _, _ = AF.affine_residuals(P, P.layout(0), gn.poses, gn.d, gn.ab)
    assert np.abs(r[gn.frozen & valid]).max() < 1e-6


def test_brightness_model_beats_the_plain_fc_on_a_brightened_scene():
    # from the true geometry with the brightness unknown (a = b = 0 to start):
    # the joint iteration finds the brightness and drops to the scene's own
    # interpolation floor; the plain model can only bend the geometry
    from oracle.gn import GaussNewton
    sc = scenes.tiny()
    ab = seeded_ab(sc.n_frames, 6)
    P = _problem(sc, brighten(sc.images, ab), sc.poses_gt, sc.inv_depth_gt)
    plain = GaussNewton(P, "fc")
    plain.iterate(0, 8)
    aff = AF.AffineFC(P)
    aff.iterate(0, 8)
    assert aff.history[-1]["rmse"] < 0.5 * plain.history[-1]["rmse"]
    assert np.abs(aff.ab - ab).max() < 2e-2


@pytest.mark.parametrize("f", [1, 3])
def test_affine_drop_equals_reduced_problem(f):
    # dropping a frame's observations equals solving the problem whose input
    # lacks them (frames and points kept), a path that shares none of the
    # drop's code: the same statistics and steps
    from tests.test_oracle_dynamic import reduced_scene_arrays
    sc = scenes.tiny()
    ab = seeded_ab(sc.n_frames, 6)
    img = brighten(sc.images, ab)
    a = AF.AffineFC(_problem(sc, img, sc.poses_gt, sc.inv_depth_gt))
    a.drop_frame(f)
    ptr, frames = reduced_scene_arrays(sc, f)
    b = AF.AffineFC(Problem(img, sc.intrinsics, sc.poses_gt, sc.host_frame, sc.host_uv, sc.inv_depth_gt, ptr,
                            frames, sc.pattern, n_levels=sc.n_levels, huber_k=sc.huber_k))
    for sa, sb in zip(a.iterate(0, 3), b.iterate(0, 3)):
        assert sa["n_active"] == sb["n_active"]
        assert abs(sa["energy"] / sb["energy"] - 1) <= 1e-12
        assert abs(sa["max_disp_px"] - sb["max_disp_px"]) <= 1e-9 * max(1.0, sb["max_disp_px"])
    np.testing.assert_allclose(a.poses, b.poses, rtol=0, atol=1e-11)
    np.testing.assert_allclose(a.d, b.d, rtol=1e-10)
    np.testing.assert_allclose(a.ab, b.ab, rtol=0, atol=1e-11)
