"""Pins of the front-end oracle (corners, tracking, geometric bundle adjustment;
the base solution of Sec. 4.1) against closed forms, invariants and the
problem's exact minimum, never against the oracle's own formulas."""
import numpy as np
import pytest

import scenes
from oracle import frontend as FE
from oracle import geometry as G
from oracle import image as IM
from oracle import solver as SV


# ------------------------------------------------------------------ corners

def test_constant_image_has_zero_response_and_no_corner():
    img = np.full((40, 50), 0.37, np.float32)
    assert not FE.harris_response(img).any()
    uv, resp = FE.detect_corners(img, cell=8, margin=8)
    assert uv.shape == (0, 2)


def test_ramp_response_is_the_closed_form():
    # q = a u + b v exactly: the gradients (times two) are 2a, 2b at every
    # pixel, the 5x5 sums 100 a^2, 100 b^2, 100 ab, det = 0, so
    # R = 16 det - tr^2 = -(100 (a^2 + b^2))^2 on the defined region
    a, b = 3, 2
    v, u = np.mgrid[0:30, 0:40]
    img = ((a * u + b * v) / np.float32(255.0)).astype(np.float32)
    assert (FE.quantize8(img) == a * u + b * v).all()
    R = FE.harris_response(img)
    inner = R[3:-3, 3:-3]
    assert (inner == -(100 * (a * a + b * b)) ** 2).all()
    assert not R[:3].any() and not R[-3:].any() and not R[:, :3].any() and not R[:, -3:].any()


def test_response_is_symmetric_under_transposition():
    rng = np.random.default_rng(0)
    img = rng.random((33, 41)).astype(np.float32)
    assert np.array_equal(FE.harris_response(img.T.copy()), FE.harris_response(img).T)


def test_square_corners_are_the_strongest():
    img = np.full((64, 80), 0.1, np.float32)
    img[20:44, 30:56] = 0.8
    uv, resp = FE.detect_corners(img, cell=4, margin=8, max_corners=4)
    assert uv.shape == (4, 2)
    got = sorted(map(tuple, uv.tolist()))
    # the square spans columns 30..55 and rows 20..43; its corner pixels
    want = [(30, 20), (30, 43), (55, 20), (55, 43)]
    for g, w in zip(got, want):
        assert abs(g[0] - w[0]) <= 1 and abs(g[1] - w[1]) <= 1, (got, want)
    # the four corners of the square respond alike (mirror images)
    assert resp.max() - resp.min() <= resp.max() // 1000 + 1


def test_plateau_keeps_its_first_pixel_and_cells_keep_one_corner():
    R = np.zeros((20, 20), np.int64)
    R[9, 9] = R[9, 10] = R[10, 9] = 50   # plateau: raster-first (9, 9) wins
    R[5, 14] = 70                         # another cell
    R[5, 15] = 60                         # same cell as (5, 14), smaller
    cand = FE.local_maxima(R, 4, 0)
    assert sorted(zip(*np.nonzero(cand))) == [(5, 14), (9, 9)]


def test_corner_order_strongest_first_then_raster():
    rng = np.random.default_rng(1)
    img = rng.random((96, 96)).astype(np.float32)
    uv, resp = FE.detect_corners(img, cell=8, margin=8, max_corners=50)
    assert uv.shape[0] == 50
    assert (np.diff(resp) <= 0).all()
    # at most one corner per cell, all inside the margin, all local maxima
    cells = (uv[:, 1] // 8) * 12 + uv[:, 0] // 8
    assert np.unique(cells).size == cells.size
    assert (uv >= 8).all() and (uv <= 96 - 9).all()
    R = FE.harris_response(img)
    for u, v in uv:
        nb = R[v - 1: v + 2, u - 1: u + 2]
        assert R[v, u] == nb.max()


# ------------------------------------------------------------------ tracking

def _smooth(width, height, shift=(0.0, 0.0)):
    """A smooth analytic image sampled at pixel centres, translated by shift."""
    v, u = np.mgrid[0:height, 0:width].astype(float)
    u = u - shift[0]
    v = v - shift[1]
    return (0.5 + 0.18 * np.sin(0.21 * u + 0.3) * np.cos(0.17 * v - 0.2)
            + 0.12 * np.sin(0.13 * u + 0.11 * v + 1.0) + 0.08 * np.cos(0.09 * u - 0.23 * v))


def _pyr(images, levels):
    pyr = IM.pyramid(np.asarray(images, np.float32), levels)
    return pyr, [IM.central_gradients(p) for p in pyr]


def _bilinear_surface(width, height, shift=(0.0, 0.0)):
    """I = a + b u + c v + e u v, translated by shift: bilinear interpolation,
    central differences and the 2x2 pyramid reproduce it exactly."""
    v, u = np.mgrid[0:height, 0:width].astype(float)
    u = u - shift[0]
    v = v - shift[1]
    return 0.1 + 0.002 * u + 0.002 * v + 0.00004 * u * v


def test_known_translation_is_recovered_exactly_on_a_bilinear_surface():
    # the model is exact, so LK converges to the shift up to the float32
    # rounding of the images
    s = (2.37, -1.61)
    pyr, grads = _pyr([_bilinear_surface(96, 80), _bilinear_surface(96, 80, s)], 3)
    xs = np.array([[40.0, 40.0], [48.0, 36.0], [56.5, 44.25]])
    # (its gradient varies slowly, so H is nearly rank one: no texture floor)
    pos, st, fb = FE.track(pyr, grads, np.zeros(3, int), xs, np.ones(3, int), xs, radius=4, n_iters=10,
                           min_eig=0.0)
    assert (st == FE.TRACK_OK).all()
    assert np.abs(pos - xs - np.array(s)).max() < 1e-4
    assert fb.max() < 1e-4


def test_known_translation_of_a_textured_image():
    # a smooth texture: bilinear sampling biases the answer by a few hundredths
    s = (2.37, -1.61)
    pyr, grads = _pyr([_smooth(128, 96), _smooth(128, 96, s)], 3)
    xs = np.array([[40.0, 40.0], [64.0, 48.0], [80.0, 50.0], [50.0, 60.0]])
    pos, st, fb = FE.track(pyr, grads, np.zeros(4, int), xs, np.ones(4, int), xs, radius=4, n_iters=10)
    assert (st == FE.TRACK_OK).all()
    assert np.abs(pos - xs - np.array(s)).max() < 0.1
    assert fb.max() < 0.1


def test_identical_images_return_to_the_start():
    pyr, grads = _pyr([_smooth(96, 80), _smooth(96, 80)], 2)
    xs = np.array([[40.0, 40.0], [48.5, 36.25]])
    pos, st, fb = FE.track(pyr, grads, [0, 0], xs, [1, 1], xs + np.array([0.8, -0.6]), radius=4, n_iters=12)
    assert (st == FE.TRACK_OK).all()
    assert np.abs(pos - xs).max() < 1e-6


def test_lost_tracks_are_flagged():
    flat = np.full((80, 96), 0.4)
    pyr, grads = _pyr([flat, flat], 1)
    xs = np.array([[40.0, 40.0]])
    _, st, _ = FE.track(pyr, grads, [0], xs, [1], xs)
    assert st[0] == FE.TRACK_LOW_TEXTURE
    pyr, grads = _pyr([_smooth(96, 80), _smooth(96, 80)], 1)
    _, st, _ = FE.track(pyr, grads, [0], xs, [1], np.array([[93.0, 40.0]]))
    assert st[0] == FE.TRACK_LEFT_IMAGE
    # a track into an unrelated image fails the forward-backward check
    rng = np.random.default_rng(3)
    other = rng.random((80, 96))
    pyr, grads = _pyr([_smooth(96, 80), other], 1)
    _, st, fb = FE.track(pyr, grads, [0, 0, 0], np.array([[40.0, 40.0], [30.0, 50.0], [60.0, 30.0]]), [1, 1, 1],
                         np.array([[40.0, 40.0], [30.0, 50.0], [60.0, 30.0]]), fb_px=0.05)
    assert (st != FE.TRACK_OK).any()


# ------------------------------------------------------------------ geometric BA

def _geo_problem(noise_px=0.0, seed=0):
    sc = scenes.tiny()
    L = FE._GeoLayout(sc.n_frames, sc.intrinsics, sc.host_frame.astype(np.int64), sc.host_uv.astype(float),
                      sc.obs_ptr.astype(np.int64), sc.obs_frame)
    from oracle import residuals as RS
    z, ok = RS.centre_pixels(L, sc.poses_gt, sc.inv_depth_gt)
    assert ok.all()
    z = z + np.random.default_rng(seed).normal(scale=noise_px, size=z.shape) if noise_px else z
    return sc, z


def test_geometric_jacobian_matches_finite_differences():
    sc, z = _geo_problem()
    ba = FE.GeometricBA(sc.intrinsics, sc.poses_init, sc.host_frame, sc.host_uv, sc.inv_depth_init, sc.obs_ptr,
                        sc.obs_frame, z)
    e0, _, act, _, _, J = ba._rows()
    A, B = SV.pair_maps(ba.L, ba.poses)
    Jabs = SV.absolute_jacobian(ba.L, J.reshape(-1, 7), A, B, sc.n_frames, sc.n_points).toarray()
    rng = np.random.default_rng(7)
    cols = list(rng.choice(6 * sc.n_frames, 12, replace=False)) + list(6 * sc.n_frames + rng.choice(sc.n_points, 6))
    h = 1e-6
    R, t = G.unpack(ba.poses)
    for c in cols:
        num = []
        for sgn in (1.0, -1.0):
            dp = np.zeros(6 * sc.n_frames)
            dd = np.zeros(sc.n_points)
            if c < 6 * sc.n_frames:
                dp[c] = sgn * h
            else:
                dd[c - 6 * sc.n_frames] = sgn * h
            d6 = dp.reshape(-1, 6)
            Rn, tn = G.boxplus_pose(R, t, d6[:, :3], d6[:, 3:])
            e, _ = ba.reprojection(G.pack(Rn, tn), ba.d + dd)
            num.append(e.reshape(-1))
        fd = (num[0] - num[1]) / (2 * h)
        assert np.allclose(Jabs[:, c], fd, rtol=1e-5, atol=1e-5 * np.abs(fd).max() + 1e-9), c


def test_noise_free_tracks_are_fitted_exactly():
    sc, z = _geo_problem()
    ba = FE.GeometricBA(sc.intrinsics, sc.poses_init, sc.host_frame, sc.host_uv, sc.inv_depth_init, sc.obs_ptr,
                        sc.obs_frame, z, huber_px=2.0)
    assert ba.step()["rmse"] > 0.05
    ba.run(30, 1e-9)
    e, ok = ba.reprojection()
    # the minimum of the reprojection energy is zero (at the ground truth up to
    # the free scale of the scene)
    assert ok.all() and np.abs(e).max() < 1e-7


def test_outliers_are_the_ones_removed():
    sc, z = _geo_problem(noise_px=0.05, seed=4)
    rng = np.random.default_rng(5)
    # gross errors on observations of points seen at least three times (a
    # point with one or two observations can fit a wrong one)
    cnt = np.diff(sc.obs_ptr)
    pool = np.nonzero(np.repeat(cnt, cnt) >= 3)[0]
    bad = rng.choice(pool, z.shape[0] // 20, replace=False)
    z = z.copy()
    z[bad] += rng.choice([-1.0, 1.0], size=(bad.size, 2)) * rng.uniform(15.0, 25.0, size=(bad.size, 2))
    ba = FE.GeometricBA(sc.intrinsics, sc.poses_init, sc.host_frame, sc.host_uv, sc.inv_depth_init, sc.obs_ptr,
                        sc.obs_frame, z, huber_px=1.0)
    iters = ba.solve(30, 1e-6, outlier_px=3.0)
    assert len(iters) == 2
    removed = set(np.nonzero(~ba.inlier)[0].tolist())
    assert set(bad.tolist()) <= removed
    assert len(removed) - bad.size <= z.shape[0] // 100
    e, _ = ba.reprojection()
    n = np.hypot(e[:, 0], e[:, 1])[ba.inlier]
    assert np.sqrt(np.mean(n * n)) < 0.1    # the inliers' noise level (0.05 px per axis)
