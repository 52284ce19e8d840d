"""GPU parity of the front end (Sec. 4.1 base solution: corners, tracks,
geometric bundle adjustment) against oracle/frontend.py, through the C ABI.

Corners are exact integer work: bit-exact. Tracks are FP64 on both sides:
positions to 1e-8 px and the same status, except where the oracle's
deciding quantity lies within rounding of a threshold. The geometric BA
runs the FC iteration in FP64: iterates to the oracle's FP64 bars."""
import numpy as np
import pytest

import scenes
from oracle import frontend as FE
from oracle import image as IM
from oracle import residuals as RS
from tests.oracle_refs import rot_err, trans_rel_err

pytestmark = pytest.mark.gpu

pba = pytest.importorskip("paper_1704_06967_amd.pba")


@pytest.fixture(scope="module")
def mid_small():
    return scenes.mid(n_per_host=300)


def frames_ctx(sc, precision=pba.PBA_FP64, mode=pba.PBA_FC, n_levels=None):
    s = pba.Solver(mode=mode, precision=precision, n_levels=sc.n_levels if n_levels is None else n_levels,
                   pattern=sc.pattern, huber_k=sc.huber_k)
    s.set_frames(sc.images, sc.intrinsics, sc.poses_init)
    return s


# ------------------------------------------------------------------ corners

@pytest.mark.parametrize("precision", [pba.PBA_FP64, pba.PBA_FP32])
@pytest.mark.parametrize("frame,cell,K", [(0, 8, 2000), (7, 8, 300), (29, 16, 5000), (3, 7, 1), (12, 8, 0)])
def test_corners_bit_exact(mid_small, precision, frame, cell, K):
    sc = mid_small
    s = frames_ctx(sc, precision)
    print(f"corners: frame {frame} cell {cell} K {K} precision {precision}", flush=True)
    uv, resp = s.corners(frame, cell=cell, margin=8, max_corners=K)
    ouv, oresp = FE.detect_corners(sc.images[frame], cell=cell, margin=8, max_corners=K)
    assert uv.shape == ouv.shape
    assert np.array_equal(uv, ouv) and np.array_equal(resp, oresp)
    s.close()


def test_corner_thresholds_and_limits(mid_small):
    sc = mid_small
    s = frames_ctx(sc)
    img = sc.images[5]
    R = FE.harris_response(img)
    thr = int(np.percentile(R[R > 0], 90))
    uv, resp = s.corners(5, cell=8, margin=20, min_response=thr, max_corners=100000 // 8)
    ouv, oresp = FE.detect_corners(img, cell=8, margin=20, min_response=thr, max_corners=100000 // 8)
    assert np.array_equal(uv, ouv) and np.array_equal(resp, oresp)
    assert (resp > thr).all() and (uv >= 20).all()
    # more cells than one call takes, and bad ranges, are refused before device work
    with pytest.raises(pba.PbaError):
        s.corners(5, cell=2)          # 320 x 240 cells
    with pytest.raises(pba.PbaError):
        s.corners(5, cell=17)
    with pytest.raises(pba.PbaError):
        s.corners(30)
    s.close()


# ------------------------------------------------------------------ tracks

def _guesses(sc, rng, err_px):
    """Level-0 positions of scene points in their targets from the true
    parameters, perturbed by err_px: the caller's prediction."""
    L = FE._GeoLayout(sc.n_frames, sc.intrinsics, sc.host_frame.astype(np.int64), sc.host_uv.astype(float),
                      sc.obs_ptr.astype(np.int64), sc.obs_frame)
    q, _ = RS.centre_pixels(L, sc.poses_gt, sc.inv_depth_gt)
    return q + rng.uniform(-err_px, err_px, size=q.shape), L


@pytest.mark.parametrize("precision,tol", [(pba.PBA_FP64, 1e-8), (pba.PBA_FP32, 2e-4)])
def test_tracks_match_the_oracle(mid_small, precision, tol):
    sc = mid_small
    rng = np.random.default_rng(11)
    guess, L = _guesses(sc, rng, 3.0)
    sel = rng.choice(L.obs_point.size, 600, replace=False)
    host = L.obs_host[sel]
    tgt = L.obs_target[sel]
    xs = sc.host_uv[L.obs_point[sel]].astype(float)
    g = guess[sel]
    # a few that start outside the image and a few with a long radius
    g[:5] = np.array([[-40.0, 10.0]] * 5)
    s = frames_ctx(sc, precision)
    print(f"tracks: {sel.size} of the mid scene, precision {precision}", flush=True)
    pos, st, fb = s.track(host, xs, tgt, g, radius=4, n_iters=10, min_eig=1e-6, fb_px=0.5)
    pyr = IM.pyramid(np.asarray(sc.images, np.float32), sc.n_levels)
    grads = [IM.central_gradients(p) for p in pyr]
    opos, ost, ofb = FE.track(pyr, grads, host, xs, tgt, g, radius=4, n_iters=10, min_eig=1e-6, fb_px=0.5)
    both = (st == FE.TRACK_OK) & (ost == FE.TRACK_OK)
    err = np.abs(pos - opos)[both].max()
    print(f"  ok {int((ost == 0).sum())} of {sel.size}; status differs {int((st != ost).sum())}; "
          f"max position difference {err:.2e} px", flush=True)
    assert (st[:5] == FE.TRACK_LEFT_IMAGE).all()
    # (targets up to 36 degrees away: many windows change too much to track)
    assert (ost == FE.TRACK_OK).sum() > sel.size // 3
    assert err <= tol
    # status may differ only where the forward-backward distance sits at the
    # threshold within the positions' agreement
    diff = st != ost
    assert (np.abs(ofb[diff] - 0.5) <= 100 * tol).all(), (st[diff], ost[diff], ofb[diff])
    s.close()


def test_track_radius_and_iterations(mid_small):
    sc = mid_small
    rng = np.random.default_rng(12)
    guess, L = _guesses(sc, rng, 2.0)
    sel = rng.choice(L.obs_point.size, 100, replace=False)
    args = (L.obs_host[sel], sc.host_uv[L.obs_point[sel]].astype(float), L.obs_target[sel], guess[sel])
    s = frames_ctx(sc)
    pyr = IM.pyramid(np.asarray(sc.images, np.float32), sc.n_levels)
    grads = [IM.central_gradients(p) for p in pyr]
    for radius, iters in [(1, 3), (5, 20), (pba.PBA_FE_MAX_RADIUS, 1)]:
        pos, st, fb = s.track(*args, radius=radius, n_iters=iters, min_eig=1e-7, fb_px=1.0)
        opos, ost, ofb = FE.track(pyr, grads, *args, radius=radius, n_iters=iters, min_eig=1e-7, fb_px=1.0)
        both = (st == 0) & (ost == 0)
        assert both.sum() > 0
        assert np.abs(pos - opos)[both].max() <= 1e-8
        assert ((st == ost) | (np.abs(ofb - 1.0) <= 1e-6)).all()
    with pytest.raises(pba.PbaError):
        s.track(*args, radius=pba.PBA_FE_MAX_RADIUS + 1)
    s.close()


# ------------------------------------------------------------------ geometric BA

def _tracks(sc, noise_px, n_bad, seed):
    L = FE._GeoLayout(sc.n_frames, sc.intrinsics, sc.host_frame.astype(np.int64), sc.host_uv.astype(float),
                      sc.obs_ptr.astype(np.int64), sc.obs_frame)
    z, ok = RS.centre_pixels(L, sc.poses_gt, sc.inv_depth_gt)
    rng = np.random.default_rng(seed)
    z = z + rng.normal(scale=noise_px, size=z.shape)
    cnt = np.diff(sc.obs_ptr)
    pool = np.nonzero(np.repeat(cnt, cnt) >= 3)[0]
    bad = rng.choice(pool, n_bad, replace=False)
    z[bad] += rng.choice([-1.0, 1.0], size=(n_bad, 2)) * rng.uniform(10.0, 20.0, size=(n_bad, 2))
    return z


@pytest.mark.parametrize("precision", [pba.PBA_FP64, pba.PBA_FP32])
@pytest.mark.parametrize("scene", ["tiny", "mid"])
def test_geometric_ba_matches_the_oracle(mid_small, precision, scene):
    sc = scenes.tiny() if scene == "tiny" else mid_small
    z = _tracks(sc, 0.1, sc.n_obs // 25, 3)
    s = frames_ctx(sc, precision)
    s.set_points(sc.host_frame, sc.host_uv, sc.inv_depth_init, sc.obs_ptr, sc.obs_frame)
    with pytest.raises(pba.PbaError):
        s.geo_solve(5)               # no tracks yet
    with pytest.raises(pba.PbaError):
        s.set_tracks(z[:-1])         # one per observation
    s.set_tracks(z)
    print(f"geometric BA: {scene}, {sc.n_obs} observations, precision {precision}", flush=True)
    res, status, inl = s.geo_solve(20, conv_px=1e-4, huber_px=1.5, outlier_px=3.0)
    ba = FE.GeometricBA(sc.intrinsics, sc.poses_init, sc.host_frame, sc.host_uv, sc.inv_depth_init, sc.obs_ptr,
                        sc.obs_frame, z, huber_px=1.5)
    iters = ba.solve(20, 1e-4, outlier_px=3.0)
    poses, d = s.get_params()
    e_rot, e_tr = rot_err(poses, ba.poses).max(), trans_rel_err(poses, ba.poses).max()
    e_d = np.abs(d / ba.d - 1).max()
    e_o, _ = ba.reprojection()
    n = np.hypot(e_o[:, 0], e_o[:, 1])[ba.inlier]
    print(f"  iters {list(res.iters[:2])} vs {iters}; rot {e_rot:.2e} trans {e_tr:.2e} inv depth {e_d:.2e}; "
          f"rmse {res.final_rmse:.4f} vs {np.sqrt(np.mean(n * n)):.4f} px", flush=True)
    assert status == pba.PBA_OK and res.converged
    assert list(res.iters[:2]) == iters
    assert np.array_equal(inl.astype(bool), ba.inlier)
    assert e_rot <= 1e-9 and e_tr <= 1e-9 and e_d <= 1e-8
    assert res.final_active == int(ba.inlier.sum())
    assert abs(res.final_rmse / np.sqrt(np.mean(n * n)) - 1) <= 1e-9
    s.close()


def test_geometric_ba_leaves_the_photometric_context_usable(mid_small):
    """After the geometric solve an IC context's photometric iterations run
    from the geometric result, as the oracle's from the same parameters."""
    from oracle.gn import GaussNewton, Problem
    sc = mid_small
    z = _tracks(sc, 0.1, 0, 5)
    s = frames_ctx(sc, pba.PBA_FP64, mode=pba.PBA_IC_PROXY)
    s.set_points(sc.host_frame, sc.host_uv, sc.inv_depth_init, sc.obs_ptr, sc.obs_frame)
    s.set_tracks(z)
    s.geo_solve(20, conv_px=1e-4, huber_px=1.5)
    poses, d = s.get_params()
    st = s.iterate(0, 2)
    prob = Problem(sc.images, sc.intrinsics, poses, sc.host_frame, sc.host_uv, d, sc.obs_ptr, sc.obs_frame,
                   sc.pattern, n_levels=sc.n_levels, huber_k=sc.huber_k)
    ost = GaussNewton(prob, "ic").iterate(0, 2)
    for a, o in zip(st, ost):
        assert a["n_active"] == o["n_active"]
        assert abs(a["energy"] / o["energy"] - 1) <= 1e-9
    s.close()
