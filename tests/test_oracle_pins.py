"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: identities
stated in the paper, closed forms, finite differences, library routines, or
the exact planar problem where bilinear interpolation and central differences
are exact.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.ndimage as ndi
from scipy.spatial.transform import Rotation

import scenes
from scenes.planar import planar
from oracle import geometry as G
from oracle import image as IM
from oracle import residuals as RS
from oracle import solver as SV
from oracle.gn import GaussNewton, Problem

RNG = np.random.default_rng(1234)


def rand_pose(rng, ang=0.3, trans=0.5):
    R = Rotation.from_rotvec(rng.normal(size=3) * ang).as_matrix()
    return R, rng.normal(size=3) * trans


def rand_points(rng, n):
    return rng.uniform(-0.4, 0.4, size=(n, 2))


# ---------------------------------------------------------------- geometry


def test_so3_exp_matches_scipy_rotvec():
    w = RNG.normal(size=(50, 3)) * np.array([[1.0], [1e-9]]).repeat(25, 0)
    np.testing.assert_allclose(G.so3_exp(w), Rotation.from_rotvec(w).as_matrix(), atol=1e-14)


def test_identity_warp_for_any_depth():
    """Sec. 3.1: with R = I, t = 0 the warp is the identity whatever d is."""
    x = rand_points(RNG, 20)
    d = RNG.uniform(0.01, 5.0, 20)
    W = G.warp(x, np.broadcast_to(np.eye(3), (20, 3, 3)), np.zeros((20, 3)), d)
    np.testing.assert_allclose(W, x, atol=1e-15)


def test_ordinary_ic_depth_derivative_is_zero():
    """Sec. 3.1 / Fig. 1: at the identity warp d W / d d = t0 = 0."""
    x = rand_points(RNG, 20)
    J = G.ordinary_ic_dW(x, RNG.uniform(0.1, 2.0, 20))
    assert np.all(J[..., 6] == 0.0)
    assert np.all(np.abs(J[..., :6]).sum(-1) > 0)


def _proxy_setup(rng, n=16):
    R0, t0 = rand_pose(rng)
    x = rand_points(rng, n)
    d0 = rng.uniform(0.2, 0.8, n)
    return x, np.broadcast_to(R0, (n, 3, 3)).copy(), np.broadcast_to(t0, (n, 3)).copy(), d0


def test_proxy_phi_identity_at_zero():
    """eq:phi / eq:phi0: phi(x; 0) = x."""
    x, R0, t0, d0 = _proxy_setup(RNG)
    np.testing.assert_allclose(G.proxy_phi0(x, R0, t0, d0, np.zeros((16, 7))), x, atol=1e-13)
    np.testing.assert_allclose(G.proxy_phi_grad_form(x, R0, t0, d0, np.zeros((16, 7))), x, atol=1e-13)
    np.testing.assert_allclose(G.proxy_phi_update_form(x, R0, t0, d0, np.zeros((16, 7))), x, atol=1e-13)


def test_proxy_phi_forms_agree():
    """eq:phi0 and eq:phi_grad are the same function for every dp."""
    x, R0, t0, d0 = _proxy_setup(RNG)
    dp = RNG.normal(size=(16, 7)) * np.array([0.05] * 6 + [0.02])
    np.testing.assert_allclose(G.proxy_phi0(x, R0, t0, d0, dp), G.proxy_phi_grad_form(x, R0, t0, d0, dp),
                               rtol=1e-12, atol=1e-13)


def test_proxy_phi_is_template_of_warp():
    """eq:phi_a: phi(x; dp) is the target point W(x; dp boxplus p(0)) taken back
    into the template through the inverse of W(.; p(0)); that inverse places the
    point on the target ray at the depth z0bar it has under p(0). Rebuild it
    from that definition with 3-D points."""
    x, R0, t0, d0 = _proxy_setup(RNG)
    dp = RNG.normal(size=(16, 7)) * 0.03
    Rp = G.so3_exp(dp[:, :3]) @ R0
    tp = t0 + dp[:, 3:6]
    dd = d0 + dp[:, 6]
    y = G.warp(x, Rp, tp, dd)  # target point with the incremented parameters
    zb = G.proxy_zbar0(x, R0, t0, d0)
    X_target = zb[:, None] * G.homog(y)  # on the ray of y at the depth z0bar
    X_template = np.einsum("nji,nj->ni", R0, X_target - t0)
    np.testing.assert_allclose(G.project(X_template), G.proxy_phi0(x, R0, t0, d0, dp), rtol=1e-12, atol=1e-13)


def test_phi_star_closed_forms():
    """Sec. 3.4: phi*(x; 0) = z0bar x~ and d phi*/d dd = M t0."""
    x, R0, t0, d0 = _proxy_setup(RNG)
    zb = G.proxy_zbar0(x, R0, t0, d0)
    np.testing.assert_allclose(G.proxy_phi_star(x, R0, t0, d0, np.zeros((16, 7))), zb[:, None] * G.homog(x),
                               rtol=1e-12)
    h = 1e-6
    e = np.zeros((16, 7))
    e[:, 6] = h
    fd = (G.proxy_phi_star(x, R0, t0, d0, e) - G.proxy_phi_star(x, R0, t0, d0, -e)) / (2 * h)
    Mt0 = np.einsum("nij,nj->ni", G.proxy_M(R0, t0, zb), t0)
    np.testing.assert_allclose(fd, Mt0, rtol=1e-8, atol=1e-10)


def test_proxy_jacobian_matches_finite_differences():
    """All 7 columns of d phi / d dp (Sec. 3.4 closed form) vs central
    differences of eq:phi0."""
    x, R0, t0, d0 = _proxy_setup(RNG)
    J = G.proxy_dphi(x, R0, t0, d0)
    h = 1e-6
    for k in range(7):
        e = np.zeros((16, 7))
        e[:, k] = h
        fd = (G.proxy_phi0(x, R0, t0, d0, e) - G.proxy_phi0(x, R0, t0, d0, -e)) / (2 * h)
        np.testing.assert_allclose(J[:, :, k], fd, rtol=1e-6, atol=1e-8, err_msg=f"column {k}")


def test_proxy_depth_derivative_quotient_rule_and_zero_iff_t0_zero():
    """Sec. 3.4: d phi / d dd = (1/phi*_z^2)[(m_x.t0) phi*_z - phi*_x (m_z.t0); ...],
    non-zero for t0 != 0 and zero for t0 = 0."""
    x, R0, t0, d0 = _proxy_setup(RNG)
    zb = G.proxy_zbar0(x, R0, t0, d0)
    M = G.proxy_M(R0, t0, zb)
    ps = G.proxy_phi_star(x, R0, t0, d0, np.zeros((16, 7)))
    mt = np.einsum("nij,nj->ni", M, t0)
    expect = np.stack([mt[:, 0] * ps[:, 2] - ps[:, 0] * mt[:, 2], mt[:, 1] * ps[:, 2] - ps[:, 1] * mt[:, 2]], 1)
    expect /= ps[:, 2:3] ** 2
    J = G.proxy_dphi(x, R0, t0, d0)
    np.testing.assert_allclose(J[:, :, 6], expect, rtol=1e-12, atol=1e-14)
    assert np.all(np.abs(J[:, :, 6]).sum(1) > 1e-6)
    J0 = G.proxy_dphi(x, R0, np.zeros_like(t0), d0)
    assert np.all(J0[:, :, 6] == 0.0)


def test_fc_warp_jacobian_matches_finite_differences():
    x = rand_points(RNG, 16)
    R, t = rand_pose(RNG)
    R = np.broadcast_to(R, (16, 3, 3)).copy()
    t = np.broadcast_to(t + np.array([0, 0, 2.0]), (16, 3)).copy()
    d = RNG.uniform(0.2, 0.8, 16)
    J = G.warp_dW(x, R, t, d)
    h = 1e-6
    for k in range(7):
        e = np.zeros((16, 7))
        e[:, k] = h

        def W(s):
            Rn, tn = G.boxplus_pose(R, t, s * e[:, :3], s * e[:, 3:6])
            return G.warp(x, Rn, tn, d + s * e[:, 6])

        np.testing.assert_allclose(J[:, :, k], (W(1) - W(-1)) / (2 * h), rtol=1e-6, atol=1e-8)


def test_absolute_maps_match_finite_differences():
    """d theta_rel = A d theta_f + B d theta_h for R_fh = R_f R_h^T,
    t_fh = t_f - R_fh t_h under left increments of the absolute poses."""
    Rf, tf = rand_pose(RNG)
    Rh, th = rand_pose(RNG)
    Rfh, tfh = G.relative_pose(Rf, tf, Rh, th)
    A, B = G.abs_maps(Rfh, th)
    h = 1e-6
    for which, Mref in (("f", A), ("h", B)):
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            out = []
            for s in (1, -1):
                if which == "f":
                    Rn, tn = G.boxplus_pose(Rf, tf, s * e[:3], s * e[3:])
                    R2, t2 = G.relative_pose(Rn, tn, Rh, th)
                else:
                    Rn, tn = G.boxplus_pose(Rh, th, s * e[:3], s * e[3:])
                    R2, t2 = G.relative_pose(Rf, tf, Rn, tn)
                # relative left increment: R2 = exp(dw) Rfh, t2 = tfh + dt
                dw = Rotation.from_matrix(R2 @ Rfh.T).as_rotvec()
                out.append(np.concatenate([dw, t2 - tfh]))
            np.testing.assert_allclose((out[0] - out[1]) / (2 * h), Mref[:, k], atol=1e-8)


def _canonical_update_form(x, R, t, d, R0, t0, d0, dp, keep_d0_over_d):
    """The composed warp of eq:update1 after substituting eq:phi_update for
    phi(x; -dp) and phi_z ~= 1/d0 (Sec. 3.6):
        < d0/(d' d) R R0^T R' x~ + d0/d R R0^T (t' - t0) + t >,
    with R' = dR^T R0, t' = t0 - dt, d' = d0 - dd (the parameters of p(0)
    incremented by -dp)."""
    dR = G.so3_exp(dp[:, :3])
    Rp = np.swapaxes(dR, -1, -2) @ R0
    tp = t0 - dp[:, 3:6]
    dp_ = d0 - dp[:, 6]
    RR = R @ np.swapaxes(R0, -1, -2)
    a = (d0 / (dp_ * d))[:, None] * np.einsum("nij,nj->ni", RR @ Rp, G.homog(x))
    fac = (d0 / d) if keep_d0_over_d else np.ones_like(d)
    b = fac[:, None] * np.einsum("nij,nj->ni", RR, tp - t0)
    return G.project(a + b + t)


def test_ic_update_reads_off_the_canonical_form():
    """Sec. 3.6: the parameter update is read off the canonical form of the
    composed warp. At p_k = p(0) (d = d0) W(x; p_{k+1}) reproduces that form
    exactly; away from p(0) it does so once the translation factor d0/d is
    set to 1, the approximation the paper makes there."""
    rng = np.random.default_rng(7)
    x, R0, t0, d0 = _proxy_setup(rng, 12)
    dp = rng.normal(size=(12, 7)) * np.array([0.02] * 6 + [0.01])
    Rn, tn, dn = G.ic_update(R0, t0, d0, R0, d0, dp[:, :3], dp[:, 3:6], dp[:, 6])
    np.testing.assert_allclose(G.warp(x, Rn, tn, dn),
                               _canonical_update_form(x, R0, t0, d0, R0, t0, d0, dp, True), atol=1e-13)
    Rk = G.so3_exp(rng.normal(size=(12, 3)) * 0.05) @ R0
    tk = t0 + rng.normal(size=(12, 3)) * 0.05
    dk = d0 * (1 + 0.1 * rng.normal(size=12))
    Rn, tn, dn = G.ic_update(Rk, tk, dk, R0, d0, dp[:, :3], dp[:, 3:6], dp[:, 6])
    np.testing.assert_allclose(G.warp(x, Rn, tn, dn),
                               _canonical_update_form(x, Rk, tk, dk, R0, t0, d0, dp, False), atol=1e-13)
    # the dropped factor matters: keeping d0/d gives a different warp
    assert np.abs(G.warp(x, Rn, tn, dn) - _canonical_update_form(x, Rk, tk, dk, R0, t0, d0, dp, True)).max() > 1e-5


def test_proxy_inverse_is_first_order():
    """Sec. 3.6: phi(x; dp)^{-1} ~= phi(x; -dp) to first order, so
    phi(phi(x; dp); -dp) - x is O(|dp|^2) (halving dp quarters it)."""
    rng = np.random.default_rng(8)
    x, R0, t0, d0 = _proxy_setup(rng, 12)
    base = rng.normal(size=(12, 7)) * np.array([0.02] * 6 + [0.01])
    errs = []
    for s in (1.0, 0.5, 0.25):
        y = G.proxy_phi0(x, R0, t0, d0, base * s)
        back = G.proxy_phi0(y, R0, t0, d0, -base * s)
        errs.append(np.max(np.abs(back - x)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_ic_update_rotation_is_left_update_by_conjugated_step():
    """R_{k+1} = R_k R0^T dR^T R0 equals exp(-Q dw) R_k with Q = R_k R0^T."""
    Rk, _ = rand_pose(RNG)
    R0, _ = rand_pose(RNG)
    dw = RNG.normal(size=3) * 0.1
    Rn, tn, _ = G.ic_update(Rk, np.zeros(3), np.ones(1), R0, np.ones(1), dw, np.ones(3), np.zeros(1))
    Q = Rk @ R0.T
    np.testing.assert_allclose(Rn, G.so3_exp(-Q @ dw) @ Rk, atol=1e-14)
    np.testing.assert_allclose(tn, -Q @ np.ones(3), atol=1e-14)


# ---------------------------------------------------------------- images


def test_bilinear_matches_scipy_map_coordinates():
    img = RNG.random((1, 30, 40))
    u = RNG.uniform(1, 36, 500)
    v = RNG.uniform(1, 26, 500)
    ref = ndi.map_coordinates(img[0], [v, u], order=1)
    np.testing.assert_allclose(IM.bilinear(img, np.zeros(500, int), u, v), ref, atol=1e-14)
    ui, vi = np.arange(1, 30), np.arange(1, 30) % 26 + 1
    np.testing.assert_array_equal(IM.bilinear(img, np.zeros(29, int), ui.astype(float), vi.astype(float)),
                                  img[0, vi, ui])


def test_central_gradients_match_numpy_gradient():
    img = RNG.random((2, 12, 15))
    gu, gv = IM.central_gradients(img)
    np.testing.assert_allclose(gu[:, 1:-1, 1:-1], np.gradient(img, axis=2)[:, 1:-1, 1:-1], atol=1e-15)
    np.testing.assert_allclose(gv[:, 1:-1, 1:-1], np.gradient(img, axis=1)[:, 1:-1, 1:-1], atol=1e-15)


def test_pyramid_is_box_average_and_level_pixels_consistent():
    """The box average of an affine image is that affine function at the
    coarse pixel centre mapped by (u + 0.5) / 2 - 0.5."""
    vv, uu = np.mgrid[0:16, 0:20].astype(float)
    img = (0.3 + 0.01 * uu - 0.02 * vv)[None]
    pyr = IM.pyramid(img, 3)
    for l in (1, 2):
        vl, ul = np.mgrid[0:pyr[l].shape[1], 0:pyr[l].shape[2]].astype(float)
        u0 = (ul + 0.5) * 2 ** l - 0.5
        v0 = (vl + 0.5) * 2 ** l - 0.5
        np.testing.assert_allclose(pyr[l][0], 0.3 + 0.01 * u0 - 0.02 * v0, atol=1e-14)
        np.testing.assert_allclose(IM.level_pixel(np.stack([u0, v0], -1), l), np.stack([ul, vl], -1), atol=1e-13)
    K = np.array([100.0, 90.0, 9.5, 7.5])
    Kl = IM.level_intrinsics(K, 1)
    # a ray through level-0 pixel (u0, v0) passes through its level-1 position
    x = (13.0 - K[2]) / K[0]
    np.testing.assert_allclose(Kl[0] * x + Kl[2], IM.level_pixel(13.0, 1), atol=1e-13)


# ---------------------------------------------------------------- Huber


def test_huber_closed_form():
    k = 9.0 / 255.0
    r = np.linspace(-0.2, 0.2, 4001)
    rho = RS.huber_rho(r, k)
    w = RS.huber_weight(r, k)
    # rho is C1 at |r| = k and its derivative equals w r (the IRLS weight)
    drho = np.gradient(rho, r)
    np.testing.assert_allclose(drho[2:-2], (w * r)[2:-2], atol=2e-4)
    np.testing.assert_allclose(RS.huber_rho(np.array([k]), k), 0.5 * k * k)
    assert RS.huber_weight(np.array([2 * k]), k)[0] == 0.5


# ---------------------------------------------------------------- residuals & Jacobians


@pytest.mark.parametrize("levels", [1, 3])
def test_planar_zero_residual_and_ic_equals_minus_fc(levels):
    """Exact planar problem: r == 0 at the true parameters at every level, and
    the IC proxy Jacobian equals minus the FC Jacobian (brightness constancy
    holds everywhere and the inverse warp at depth z0bar is exact on the
    fronto-parallel plane when R0 = I)."""
    sc = planar(n_levels=levels)
    P = Problem.from_scene(sc)
    for l in range(levels):
        L = P.layout(l)
        r, valid, q, _ = RS.warp_residuals(P, L, sc.poses_gt, sc.inv_depth_gt)
        assert valid.sum() > 0.9 * valid.size
        np.testing.assert_allclose(r[valid], 0.0, atol=1e-13)
        Jfc = RS.fc_jacobian(P, L, sc.poses_gt, sc.inv_depth_gt, q)
        Jic = RS.ic_jacobian(L, sc.poses_gt, sc.inv_depth_gt)
        np.testing.assert_allclose(Jic[valid], -Jfc[valid], rtol=1e-10, atol=1e-12)
        assert np.abs(Jic[valid, 6]).max() > 1e-3


def _affine_problem(scene, seed=0):
    F, H, W = scene.images.shape
    vv, uu = np.mgrid[0:H, 0:W].astype(float)
    rng = np.random.default_rng(seed)
    imgs = np.stack([0.5 + rng.normal() * 1e-3 * uu + rng.normal() * 1e-3 * vv for _ in range(F)])
    return Problem(imgs, scene.intrinsics, scene.poses_init, scene.host_frame, scene.host_uv,
                   scene.inv_depth_init, scene.obs_ptr, scene.obs_frame, scene.pattern, 1)


@pytest.fixture(scope="module")
def tiny_scene():
    return scenes.tiny(n_points=120)


def test_fc_absolute_jacobian_matches_finite_differences(tiny_scene):
    """With affine images the residual is a smooth function of p, so the FC
    Jacobian on the absolute parameters must match central differences."""
    P = _affine_problem(tiny_scene)
    L = P.layout(0)
    poses, d = P.poses_init.copy(), P.inv_depth_init.copy()
    r, valid, q, _ = RS.warp_residuals(P, L, poses, d)
    J = RS.fc_jacobian(P, L, poses, d, q)
    A, B = SV.pair_maps(L, poses)
    Jabs = SV.absolute_jacobian(L, J, A, B, P.n_frames, P.n_points).tocsc()
    h = 1e-6
    for f in range(P.n_frames):
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            out = []
            for s in (1, -1):
                R, t = G.unpack(poses)
                Rn, tn = G.boxplus_pose(R[f], t[f], s * e[:3], s * e[3:])
                pp = poses.copy()
                pp[f] = G.pack(Rn, tn)
                out.append(RS.warp_residuals(P, L, pp, d)[0])
            fd = (out[0] - out[1]) / (2 * h)
            an = Jabs[:, 6 * f + k].toarray().ravel()
            np.testing.assert_allclose(an[valid], fd[valid], atol=1e-7 * max(1e-3, np.abs(an).max()))
    dd = np.zeros_like(d)
    dd[::3] = h
    fd = (RS.warp_residuals(P, L, poses, d + dd)[0] - RS.warp_residuals(P, L, poses, d - dd)[0]) / (2 * h)
    an = Jabs[:, 6 * P.n_frames:] @ (dd / h)
    np.testing.assert_allclose(an[valid], fd[valid], atol=1e-8)


def test_ic_jacobian_matches_finite_differences_of_template_under_phi(tiny_scene):
    """J_IC = grad I0 . d phi/d dp: with an affine template, I0(phi(x; dp)) is
    smooth in dp and its central differences must match the IC row."""
    P = _affine_problem(tiny_scene, seed=3)
    L = P.layout(0)
    poses, d = P.poses_init, P.inv_depth_init
    J = RS.ic_jacobian(L, poses, d)
    Rr, tr = RS.pair_poses(L, poses)
    R0, t0, d0 = Rr[L.res_pair], tr[L.res_pair], d[L.res_point]
    h = 1e-6
    for k in range(7):
        e = np.zeros((L.x.shape[0], 7))
        e[:, k] = h
        vals = []
        for s in (1, -1):
            y = G.proxy_phi0(L.x, R0, t0, d0, s * e)
            Kh = L.Kh
            u = Kh[:, 0] * y[:, 0] + Kh[:, 2]
            v = Kh[:, 1] * y[:, 1] + Kh[:, 3]
            vals.append(IM.bilinear(P.pyr[0], L.res_host, u, v))
        fd = (vals[0] - vals[1]) / (2 * h)
        np.testing.assert_allclose(J[L.host_ok, k], fd[L.host_ok], atol=1e-8)


def test_scale_gauge_in_kernel_and_gradient_orthogonal(tiny_scene):
    """Scaling the world (t -> (1+e) t, d -> d/(1+e)) leaves every warp
    unchanged, so the vector dt_f = t_f, dd_n = -d_n lies in ker J (FC at p,
    IC at p(0)) and g = J^T W r is orthogonal to it."""
    P = Problem.from_scene(tiny_scene)
    for mode in ("fc", "ic"):
        gn = GaussNewton(P, mode)
        gn.start_level(0)
        gn.step()
        nv = np.zeros(6 * P.n_frames + P.n_points)
        for f in range(P.n_frames):
            nv[6 * f + 3:6 * f + 6] = P.poses_init[f, 9:]
        nv[6 * P.n_frames:] = -P.inv_depth_init
        if mode == "ic":
            Jabs = gn.Jabs
        else:
            L = gn.L
            r, valid, q, _ = RS.warp_residuals(P, L, P.poses_init, P.inv_depth_init)
            J = RS.fc_jacobian(P, L, P.poses_init, P.inv_depth_init, q)
            J[~valid] = 0
            A, B = SV.pair_maps(L, P.poses_init)
            Jabs = SV.absolute_jacobian(L, J, A, B, P.n_frames, P.n_points)
        Jn = Jabs @ nv
        assert np.abs(Jn).max() < 1e-12 * max(1.0, abs(Jabs).max())
        g = gn.last["g"]
        assert abs(g @ nv) < 1e-10 * np.linalg.norm(g) * np.linalg.norm(nv)


def test_schur_solve_equals_dense_full_solve():
    """Depth elimination + reduced Cholesky = the full damped, pinned system
    solved directly (FC system at p, IC system at p(0))."""
    sc = scenes.tiny(n_points=40)
    P = Problem.from_scene(sc)
    for mode in ("fc", "ic"):
        gn = GaussNewton(P, mode)
        gn.start_level(0)
        L = gn.L
        if mode == "fc":
            r, valid, q, _ = RS.warp_residuals(P, L, gn.poses, gn.d)
            J = RS.fc_jacobian(P, L, gn.poses, gn.d, q)
            J[~valid] = 0
            A, B = SV.pair_maps(L, gn.poses)
            Jabs = SV.absolute_jacobian(L, J, A, B, P.n_frames, P.n_points)
            w = RS.huber_weight(r, P.huber_k) * valid
            H, g = SV.normal_equations(Jabs, w, np.where(valid, r, 0))
        else:
            H, g = gn.H, gn.Jabs.T @ np.where(gn.frozen, 1.0, 0.0)
        red = SV.Reduced(H, P.n_frames, P.damping_rel, P.pinned_frame)
        dth, dd, _ = red.solve(g)
        dth2, dd2 = SV.dense_solve(H, g, P.n_frames, P.damping_rel, P.pinned_frame)
        np.testing.assert_allclose(dth, dth2, rtol=1e-8, atol=1e-10 * np.abs(dth2).max())
        np.testing.assert_allclose(dd, dd2, rtol=1e-8, atol=1e-10 * np.abs(dd2).max())


def test_two_host_schur_matches_dense():
    """Same check with points hosted in two different frames."""
    sc = scenes.mid(n_per_host=15, width=160, height=120, n_frames=12)
    P = Problem.from_scene(sc, n_levels=1)
    gn = GaussNewton(P, "fc")
    gn.start_level(0)
    gn.step()
    H, g = gn.last["H"], gn.last["g"]
    red = SV.Reduced(H, P.n_frames, P.damping_rel, P.pinned_frame)
    dth, dd, _ = red.solve(g)
    dth2, dd2 = SV.dense_solve(H, g, P.n_frames, P.damping_rel, P.pinned_frame)
    assert len(set(sc.host_frame.tolist())) >= 2
    np.testing.assert_allclose(dth, dth2, rtol=1e-7, atol=1e-9 * np.abs(dth2).max())
    np.testing.assert_allclose(dd, dd2, rtol=1e-7, atol=1e-9 * np.abs(dd2).max())


def test_no_huber_gn_step_equals_least_squares(tiny_scene):
    """With k = inf the weights are 1 and the GN step is the least-squares
    solution of J dp = -r with the damping rows appended and the pinned frame
    removed (scipy.linalg.lstsq)."""
    P = Problem.from_scene(tiny_scene, huber_k=np.inf)
    gn = GaussNewton(P, "fc")
    gn.start_level(0)
    poses0, d0 = gn.poses.copy(), gn.d.copy()
    gn.step()
    L = gn.L
    r, valid, q, _ = RS.warp_residuals(P, L, poses0, d0)
    J = RS.fc_jacobian(P, L, poses0, d0, q)
    J[~valid] = 0
    r = np.where(valid, r, 0.0)
    A, B = SV.pair_maps(L, poses0)
    Jabs = SV.absolute_jacobian(L, J, A, B, P.n_frames, P.n_points).toarray()
    n6 = 6 * P.n_frames
    H = Jabs.T @ Jabs
    mu_p = P.damping_rel * np.mean(np.diag(H)[:n6])
    mu_d = P.damping_rel * np.mean(np.diag(H)[n6:])
    keep = np.r_[np.arange(6, n6), np.arange(n6, Jabs.shape[1])]
    Jk = Jabs[:, keep]
    damp = np.sqrt(np.where(keep < n6, mu_p, mu_d))
    Aug = np.vstack([Jk, np.diag(damp)])
    rhs = np.concatenate([-r, np.zeros(keep.size)])
    sol = sla.lstsq(Aug, rhs)[0]
    dth = np.zeros(n6)
    dth[6:] = sol[: n6 - 6]
    dd = sol[n6 - 6:]
    np.testing.assert_allclose(gn.d - d0, dd, rtol=1e-6, atol=1e-9)
    R0, t0 = G.unpack(poses0)
    R1, t1 = G.unpack(gn.poses)
    np.testing.assert_allclose(t1 - t0, dth.reshape(-1, 6)[:, 3:], rtol=1e-6, atol=1e-11)


def test_gn_converges_on_planar_problem_from_small_perturbation():
    """On the exact planar problem (r == 0 at the truth) both FC and IC drive the
    energy to zero from a small perturbation of the poses and depths."""
    sc = planar(n_points=60, n_frames=4)
    rng = np.random.default_rng(3)
    for mode in ("fc", "ic"):
        P = Problem.from_scene(sc)
        gn = GaussNewton(P, mode)
        for f in range(1, 4):
            gn.poses[f, 9:] += rng.normal(size=3) * 1e-3
        gn.d = gn.d * (1 + 1e-3 * rng.normal(size=gn.d.shape))
        e0 = gn.evaluate(0)["energy"]
        gn.iterate(0, 8)
        e1 = gn.evaluate(0)["energy"]
        assert e1 < 1e-6 * e0, (mode, e0, e1)


def test_ic_first_iteration_step_equals_fc_step_on_planar_problem():
    """At p(0) on the exact planar problem J_IC = -J_FC, so the IC step solves
    the same system with the opposite sign, and the IC update (which composes
    with -dp) moves the parameters exactly as the FC step does to first order:
    after one iteration both land within O(|dp|^2) of each other."""
    sc = planar(n_points=60, n_frames=4)
    rng = np.random.default_rng(4)
    P = Problem.from_scene(sc)
    pert = np.zeros((4, 3))
    pert[1:] = rng.normal(size=(3, 3)) * 2e-4
    out = {}
    for mode in ("fc", "ic"):
        gn = GaussNewton(P, mode)
        gn.poses[:, 9:] += pert
        gn.iterate(0, 1)
        out[mode] = (gn.poses.copy(), gn.d.copy())
    step = np.abs(out["fc"][0][:, 9:] - (sc.poses_gt[:, 9:] + pert)).max()
    diff = np.abs(out["fc"][0] - out["ic"][0]).max()
    assert step > 1e-5 and diff < 0.05 * step, (step, diff)


# ---------------------------------------------------------------- convergence test (Sec. 4.1)


def _world_point_pixels(scene, poses, d):
    """Level-0 pixel of every observation's point centre, by another route than
    the oracle's relative-pose warp: back-project the host pixel at depth 1/d
    into world coordinates with the host's absolute pose, then project the world
    point with the target's absolute pose."""
    N = scene.n_points
    obs_point = np.repeat(np.arange(N), np.diff(scene.obs_ptr))
    K = scene.intrinsics
    h, f = scene.host_frame[obs_point], scene.obs_frame
    uv = scene.host_uv[obs_point].astype(float)
    ray = np.stack([(uv[:, 0] - K[h, 2]) / K[h, 0], (uv[:, 1] - K[h, 3]) / K[h, 1], np.ones(len(h))], 1)
    Xc = ray / d[obs_point][:, None]
    R = poses[:, :9].reshape(-1, 3, 3)
    t = poses[:, 9:]
    Xw = np.einsum("oji,oj->oi", R[h], Xc - t[h])
    Xf = np.einsum("oij,oj->oi", R[f], Xw) + t[f]
    return np.stack([K[f, 0] * Xf[:, 0] / Xf[:, 2] + K[f, 2], K[f, 1] * Xf[:, 1] / Xf[:, 2] + K[f, 3]], 1)


def _rolled_pattern(scene):
    """The scene with its patch pattern rotated so that the first pattern pixel
    is not the point centre (a test that reads a pattern pixel fails)."""
    scene.pattern = np.roll(scene.pattern, -1, axis=0)
    assert np.any(scene.pattern[0] != 0)
    return scene


def test_centre_pixels_equal_world_point_projection():
    """Several hosts, rotated and translated cameras, 3 pyramid levels: the
    centre pixel of every observation is the level-0 projection of the point's
    world position, whatever level's layout computes it."""
    sc = _rolled_pattern(scenes.mid(n_per_host=60))
    P = Problem.from_scene(sc)
    rng = np.random.default_rng(8)
    d = sc.inv_depth_init * (1 + 0.02 * rng.normal(size=sc.n_points))
    ref = _world_point_pixels(sc, sc.poses_init, d)
    for level in range(3):
        q, ok = RS.centre_pixels(P.layout(level), sc.poses_init, d)
        assert ok.all()
        np.testing.assert_allclose(q, ref, rtol=0, atol=1e-9)


def test_centre_pixels_planar_closed_form():
    """Planar problem: inverting the image generator's map (host pixel of a
    target pixel on the plane Z = Z0 under a pure translation t) gives the
    target pixel of a host pixel as c + ((u_h - c) Z0 + f t_x) / (Z0 + t_z)."""
    sc = _rolled_pattern(planar(n_levels=3, n_points=30))
    P = Problem.from_scene(sc)
    z0 = 1.0 / sc.inv_depth_gt[0]
    K = sc.intrinsics[0]
    obs_point = np.repeat(np.arange(sc.n_points), np.diff(sc.obs_ptr))
    t = sc.poses_gt[sc.obs_frame, 9:]
    uh = sc.host_uv[obs_point].astype(float)
    ref = np.stack([K[2] + ((uh[:, 0] - K[2]) * z0 + K[0] * t[:, 0]) / (z0 + t[:, 2]),
                    K[3] + ((uh[:, 1] - K[3]) * z0 + K[1] * t[:, 1]) / (z0 + t[:, 2])], 1)
    for level in range(3):
        q, ok = RS.centre_pixels(P.layout(level), sc.poses_gt, sc.inv_depth_gt)
        assert ok.all()
        np.testing.assert_allclose(q, ref, rtol=0, atol=1e-10)


def test_max_centre_displacement_of_known_translations():
    """Planar problem: moving target k by delta_k along x shifts every centre it
    observes by f delta_k / (Z0 + t_z,k) level-0 pixels (the closed form above
    is linear in t_x); the measure is the largest of these, at every level."""
    sc = planar(n_levels=3, n_frames=4, n_points=30)
    P = Problem.from_scene(sc)
    z0 = 1.0 / sc.inv_depth_gt[0]
    f = sc.intrinsics[0, 0]
    delta = np.array([0.0, 3e-4, -7e-4, 2e-4])
    moved = sc.poses_gt.copy()
    moved[:, 9] += delta
    shift = np.abs(f * delta / (z0 + sc.poses_gt[:, 11]))
    for level in range(3):
        m = RS.max_centre_displacement(P.layout(level), sc.poses_gt, sc.inv_depth_gt, moved, sc.inv_depth_gt)
        np.testing.assert_allclose(m, shift.max(), rtol=1e-9)
    # a depth change alone moves centres along their epipolar lines: compare
    # with the world-point route
    d2 = sc.inv_depth_gt * (1 + 1e-3 * np.arange(sc.n_points) / sc.n_points)
    ref = np.hypot(*(_world_point_pixels(sc, sc.poses_gt, d2) - _world_point_pixels(sc, sc.poses_gt,
                                                                                     sc.inv_depth_gt)).T).max()
    m = RS.max_centre_displacement(P.layout(2), sc.poses_gt, sc.inv_depth_gt, sc.poses_gt, d2)
    np.testing.assert_allclose(m, ref, rtol=1e-7)


@pytest.mark.parametrize("mode", ["fc", "ic"])
def test_gn_reports_displacement_of_its_own_step(mode):
    """Every Gauss-Newton iteration reports the largest level-0 displacement of
    the point centres between the parameters it started from and those it
    returns (world-point route), at every level of a 2-level solve."""
    sc = _rolled_pattern(scenes.mid(n_per_host=40))
    P = Problem.from_scene(sc, n_levels=2)
    gn = GaussNewton(P, mode)
    for level in (1, 0):
        for _ in range(2):
            before = (gn.poses.copy(), gn.d.copy())
            st = gn.iterate(level, 1)[0]
            ref = np.hypot(*(_world_point_pixels(sc, gn.poses, gn.d) - _world_point_pixels(sc, *before)).T).max()
            assert ref > 1e-4
            np.testing.assert_allclose(st["max_disp_px"], ref, rtol=1e-7)


def test_recentring_reproduces_a_fresh_level_start():
    """Proxy re-centring (Sec. 3.6: the proxy update holds near p(0)): after m
    IC iterations with recentre_every = m, the next iteration equals the first
    iteration of a fresh IC solve started (at the same level) from the
    parameters reached, bit for bit; recentre_every = 0 is the plain
    iteration."""
    sc = scenes.tiny()
    P = Problem.from_scene(sc)
    m = 2
    gr = GaussNewton(P, "ic", recentre_every=m)
    gr.iterate(0, m)
    p_m, d_m = gr.poses.copy(), gr.d.copy()
    gr.step()
    P2 = Problem(sc.images, sc.intrinsics, p_m, sc.host_frame, sc.host_uv, d_m, sc.obs_ptr, sc.obs_frame,
                 sc.pattern, n_levels=sc.n_levels, huber_k=sc.huber_k)
    fresh = GaussNewton(P2, "ic")
    fresh.iterate(0, 1)
    np.testing.assert_array_equal(gr.poses, fresh.poses)
    np.testing.assert_array_equal(gr.d, fresh.d)
    np.testing.assert_array_equal(gr.red.S, fresh.red.S)
    # without re-centring the third iteration keeps the level's first linearization
    g0 = GaussNewton(P, "ic")
    g0.iterate(0, m + 1)
    g1 = GaussNewton(P, "ic", recentre_every=0)
    g1.iterate(0, m + 1)
    np.testing.assert_array_equal(g0.poses, g1.poses)
    assert not np.array_equal(g0.poses, gr.poses)
    np.testing.assert_array_equal(g0.poses0, P.poses_init)


def test_recentring_every_iteration_matches_fc_on_the_exact_planar_problem():
    """On the exact planar problem (J_IC = -J_FC at the truth, brightness
    constancy exact) IC re-centred at every iteration converges to the truth
    like FC does: zero energy."""
    sc = planar(n_points=60, seed=3)
    P = Problem.from_scene(sc)
    g = GaussNewton(P, "ic", recentre_every=1)
    st = g.iterate(0, 8)
    assert st[-1]["energy"] < 1e-12 * max(st[0]["energy"], 1e-30) + 1e-20
