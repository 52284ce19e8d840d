"""Per-residual quantities (oracle, FP64, test infrastructure).

There is one residual per observing frame f, per point n, per patch pixel x
(Sec. 3.5): r = I0(x) - I_f(W(x; p_fn)). Each point carries one inverse depth
shared by its patch pixels (eq:energy, eq:warp). With several host frames the
paper's (R_f, t_f) is read as the pose of the target relative to the point's
host frame.
"""
import numpy as np

from . import geometry as G
from . import image as IM


class Layout:
    """Index arrays and template data of every residual at one pyramid level.

    Residual index = obs * P + j, observations in the CSR order of the input
    (point-major), j the patch pixel."""

    def __init__(self, prob, level):
        self.level = level
        P = prob.pattern.shape[0]
        N = prob.host_frame.shape[0]
        counts = np.diff(prob.obs_ptr)
        obs_point = np.repeat(np.arange(N), counts)
        self.obs_point = obs_point
        self.obs_target = prob.obs_frame.astype(np.int64)
        self.obs_host = prob.host_frame[obs_point].astype(np.int64)
        O = obs_point.shape[0]
        self.n_obs, self.P = O, P
        self.res_obs = np.repeat(np.arange(O), P)
        self.res_pat = np.tile(np.arange(P), O)
        self.res_point = obs_point[self.res_obs]
        self.res_target = self.obs_target[self.res_obs]
        self.res_host = self.obs_host[self.res_obs]
        # pairs (host, target), sorted
        key = self.obs_host * prob.n_frames + self.obs_target
        uniq, inv = np.unique(key, return_inverse=True)
        self.pair_host = uniq // prob.n_frames
        self.pair_target = uniq % prob.n_frames
        self.obs_pair = inv
        self.res_pair = inv[self.res_obs]

        stack = prob.pyr[level]
        self.H, self.W = stack.shape[1], stack.shape[2]
        Kh = IM.level_intrinsics(prob.intrinsics[self.res_host], level)
        self.Kt = IM.level_intrinsics(prob.intrinsics[self.res_target], level)
        self.Kh = Kh
        hp = IM.level_pixel(prob.host_uv[self.res_point].astype(float), level) + prob.pattern[self.res_pat]
        self.host_px = hp
        # normalized template coordinates of the patch pixel
        self.x = np.stack([(hp[:, 0] - Kh[:, 2]) / Kh[:, 0], (hp[:, 1] - Kh[:, 3]) / Kh[:, 1]], -1)
        self.host_ok = IM.in_bounds(hp[:, 0], hp[:, 1], self.W, self.H)
        gu, gv = prob.grads[level]
        self.I0 = IM.bilinear(stack, self.res_host, hp[:, 0], hp[:, 1])
        self.g0 = np.stack([IM.bilinear(gu, self.res_host, hp[:, 0], hp[:, 1]),
                            IM.bilinear(gv, self.res_host, hp[:, 0], hp[:, 1])], -1)
        # point centre (level-0 pixel, normalized with host level-0 intrinsics) for the convergence test
        K0 = prob.intrinsics[self.obs_host]
        c = prob.host_uv[obs_point].astype(float)
        self.obs_x0 = np.stack([(c[:, 0] - K0[:, 2]) / K0[:, 0], (c[:, 1] - K0[:, 3]) / K0[:, 1]], -1)
        self.obs_K0t = prob.intrinsics[self.obs_target]


def pair_poses(layout, poses):
    """Relative pose (R, t) of every pair and the absolute host translation."""
    R, t = G.unpack(poses)
    Rr, tr = G.relative_pose(R[layout.pair_target], t[layout.pair_target], R[layout.pair_host], t[layout.pair_host])
    return Rr, tr


def warp_residuals(prob, layout, poses, d):
    """Residuals at parameters (poses, d). Returns r, valid mask, target pixel q,
    transformed point v. `valid` = host patch pixel usable, d > 0, v_z > 0 and
    the target pixel usable (see image.in_bounds)."""
    Rr, tr = pair_poses(layout, poses)
    R = Rr[layout.res_pair]
    t = tr[layout.res_pair]
    dn = d[layout.res_point]
    v = G.transform(layout.x, R, t, dn)
    vz = v[:, 2]
    valid = layout.host_ok & (dn > 0) & (vz > 0)
    vzs = np.where(vz > 0, vz, 1.0)
    K = layout.Kt
    q = np.stack([K[:, 0] * v[:, 0] / vzs + K[:, 2], K[:, 1] * v[:, 1] / vzs + K[:, 3]], -1)
    valid &= IM.in_bounds(q[:, 0], q[:, 1], layout.W, layout.H)
    If = IM.bilinear(prob.pyr[layout.level], layout.res_target, q[:, 0], q[:, 1])
    r = layout.I0 - If
    return r, valid, q, v


def huber_weight(r, k):
    """IRLS weight of the Huber norm: 1 inside [-k, k], k/|r| outside."""
    a = np.abs(r)
    return np.where(a <= k, 1.0, k / np.where(a > 0, a, 1.0))


def huber_rho(r, k):
    """Huber norm ||r||_gamma (eq:energy): r^2/2 inside [-k, k], k|r| - k^2/2 outside."""
    a = np.abs(r)
    return np.where(a <= k, 0.5 * r * r, k * a - 0.5 * k * k)


def fc_jacobian(prob, layout, poses, d, q):
    """Forward-compositional Jacobian rows d r / d dp (relative pose increment
    and inverse depth) at the current parameters:
        J = -[fx g_u, fy g_v] dW/dp,
    g the target gradient interpolated at q (r = I0 - I_f(W), so dr = -dI_f)."""
    Rr, tr = pair_poses(layout, poses)
    R = Rr[layout.res_pair]
    t = tr[layout.res_pair]
    dn = d[layout.res_point]
    dW = G.warp_dW(layout.x, R, t, dn)
    gu, gv = prob.grads[layout.level]
    gqu = IM.bilinear(gu, layout.res_target, q[:, 0], q[:, 1])
    gqv = IM.bilinear(gv, layout.res_target, q[:, 0], q[:, 1])
    K = layout.Kt
    return -((K[:, 0] * gqu)[:, None] * dW[:, 0, :] + (K[:, 1] * gqv)[:, None] * dW[:, 1, :])


def ic_jacobian(layout, poses0, d0):
    """Inverse-compositional Jacobian rows with proxy templates (Sec. 3.5):
        J = grad I0 . d phi / d dp |_{dp=0},
    grad I0 at the template pixel x (host image, pixel units scaled by the host
    focal lengths), d phi / d dp from Sec. 3.4 at p(0)."""
    Rr, tr = pair_poses(layout, poses0)
    R0 = Rr[layout.res_pair]
    t0 = tr[layout.res_pair]
    dn = d0[layout.res_point]
    dphi = G.proxy_dphi(layout.x, R0, t0, dn)
    K = layout.Kh
    return (K[:, 0] * layout.g0[:, 0])[:, None] * dphi[:, 0, :] + (K[:, 1] * layout.g0[:, 1])[:, None] * dphi[:, 1, :]


def centre_pixels(layout, poses, d):
    """Level-0 pixel of each observation's point centre in its target frame and
    a flag v_z > 0 (used by the convergence test of Sec. 4.1)."""
    Rr, tr = pair_poses(layout, poses)
    R = Rr[layout.obs_pair]
    t = tr[layout.obs_pair]
    v = G.transform(layout.obs_x0, R, t, d[layout.obs_point])
    vz = v[:, 2]
    ok = vz > 0
    vzs = np.where(ok, vz, 1.0)
    K = layout.obs_K0t
    q = np.stack([K[:, 0] * v[:, 0] / vzs + K[:, 2], K[:, 1] * v[:, 1] / vzs + K[:, 3]], -1)
    return q, ok


def max_centre_displacement(layout, poses_a, d_a, poses_b, d_b, live=None):
    """Convergence measure of Sec. 4.1: the largest change, in level-0 pixels,
    of the reprojected point centres between parameters a and b, over every
    observation whose centre lies in front of the target camera under both
    (and, with `live`, that is still in the window). The measure does not
    depend on the pyramid level being iterated."""
    qa, oka = centre_pixels(layout, poses_a, d_a)
    qb, okb = centre_pixels(layout, poses_b, d_b)
    ok = oka & okb
    if live is not None:
        ok = ok & live
    disp = np.hypot(qb[:, 0] - qa[:, 0], qb[:, 1] - qa[:, 1])
    return float(np.max(np.where(ok, disp, 0.0))) if ok.size else 0.0
