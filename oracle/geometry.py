"""Geometry of the warp and of the proxy warp (oracle, FP64, test infrastructure).

Conventions
  * A pose is world->camera: X_cam = R X_world + t (Sec. 1, the SE(3) matrix
    [R t; 0 1]). Stored as 12 numbers: R row-major, then t.
  * A pose increment is the decoupled left increment (dw, dt): R <- exp(dw) R,
    t <- t + dt. The paper calls its boxplus "left multiplicative" but every
    explicit formula it writes (eq:phi, the definitions under eq:phi_update,
    phi*) uses R = dR R0, t = t0 + dt; that explicit form is the reading used.
    Parameter order of a Jacobian row: (w_x, w_y, w_z, t_x, t_y, t_z, d).
"""
import numpy as np


def skew(a):
    """[a]_x such that [a]_x b = a x b; a: [..., 3] -> [..., 3, 3]."""
    a = np.asarray(a, float)
    z = np.zeros(a.shape[:-1])
    return np.stack([
        np.stack([z, -a[..., 2], a[..., 1]], -1),
        np.stack([a[..., 2], z, -a[..., 0]], -1),
        np.stack([-a[..., 1], a[..., 0], z], -1),
    ], -2)


def so3_exp(w):
    """Rodrigues' formula exp([w]_x); w: [..., 3]."""
    w = np.asarray(w, float)
    th2 = np.sum(w * w, -1)[..., None, None]
    th = np.sqrt(th2)
    small = th2 < 1e-16
    ths = np.where(small, 1.0, th)
    a = np.where(small, 1.0 - th2 / 6.0, np.sin(ths) / ths)
    b = np.where(small, 0.5 - th2 / 24.0, (1.0 - np.cos(ths)) / (ths * ths))
    K = skew(w)
    return np.eye(3) + a * K + b * (K @ K)


def unpack(poses):
    """[..., 12] -> R [..., 3, 3], t [..., 3]."""
    poses = np.asarray(poses, float)
    return poses[..., :9].reshape(poses.shape[:-1] + (3, 3)), poses[..., 9:].copy()


def pack(R, t):
    return np.concatenate([R.reshape(R.shape[:-2] + (9,)), t], -1)


def homog(x):
    """x~ = [x^T 1]^T (Notation)."""
    x = np.asarray(x, float)
    return np.concatenate([x, np.ones(x.shape[:-1] + (1,))], -1)


def project(v):
    """<[x y z]^T> = [x/z, y/z]^T, projection onto the plane z = 1 (Notation)."""
    v = np.asarray(v, float)
    return v[..., :2] / v[..., 2:3]


def relative_pose(Rf, tf, Rh, th):
    """Pose of target f relative to host h: R = Rf Rh^T, t = tf - R th.
    With the host at the world origin (R_h = I, t_h = 0) this is exactly the
    paper's (R_f, t_f) of eq:warp."""
    R = Rf @ np.swapaxes(Rh, -1, -2)
    t = tf - np.einsum("...ij,...j->...i", R, th)
    return R, t


def transform(x, R, t, d):
    """v = R x~ + d t, the 3-D point before projection in eq:warp."""
    return np.einsum("...ij,...j->...i", R, homog(x)) + d[..., None] * t


def warp(x, R, t, d):
    """W(x; p) = <R x~ + d t> (eq. 1, eq:warp)."""
    return project(transform(x, R, t, d))


def boxplus_pose(R, t, dw, dt):
    """Forward-compositional pose increment: R <- exp(dw) R, t <- t + dt."""
    return so3_exp(dw) @ R, t + dt


def proxy_zbar0(x, R0, t0, d0):
    """z0bar: depth of the point in the target as projected by p(0)
    (the quantity under eq:phi0): v0_z / d0 with v0 = R0 x~ + d0 t0."""
    return transform(x, R0, t0, d0)[..., 2] / d0


def proxy_M(R0, t0, zbar0):
    """M = R0^T (z0bar I - [0 0 t0]) (Sec. 3.4)."""
    n = np.broadcast_shapes(np.shape(zbar0), R0.shape[:-2])
    zI = np.asarray(zbar0, float).reshape(n + (1, 1)) * np.eye(3)
    T3 = np.zeros(np.broadcast_shapes(n, t0.shape[:-1]) + (3, 3))
    T3[..., :, 2] = t0
    return np.swapaxes(R0, -1, -2) @ (zI - T3)


def _incremented(R0, t0, d0, dp):
    """p' = dp boxplus p(0): R' = exp(dw) R0, t' = t0 + dt, d' = d0 + dd."""
    dp = np.asarray(dp, float)
    return so3_exp(dp[..., 0:3]) @ R0, t0 + dp[..., 3:6], d0 + dp[..., 6]


def proxy_phi0(x, R0, t0, d0, dp):
    """phi(x; dp) in the form eq:phi0: warp x into the target with the
    incremented parameters, then back into the template through the inverse of
    W(.; p(0)), which keeps the target depth fixed at z0bar."""
    Rp, tp, dd = _incremented(R0, t0, d0, dp)
    vp = transform(x, Rp, tp, dd)
    zb = proxy_zbar0(x, R0, t0, d0)
    inner = zb[..., None] * vp / vp[..., 2:3] - t0
    return project(np.einsum("...ji,...j->...i", R0, inner))


def proxy_phi_grad_form(x, R0, t0, d0, dp):
    """phi(x; dp) = <M (R' x~ + d' t')> (eq:phi_grad)."""
    Rp, tp, dd = _incremented(R0, t0, d0, dp)
    M = proxy_M(R0, t0, proxy_zbar0(x, R0, t0, d0))
    return project(np.einsum("...ij,...j->...i", M, transform(x, Rp, tp, dd)))


def proxy_phi_star(x, R0, t0, d0, dp):
    """phi*(x; dp) = M ((dR R0) x~ + (d0 + dd)(t0 + dt)) (Sec. 3.4)."""
    Rp, tp, dd = _incremented(R0, t0, d0, dp)
    M = proxy_M(R0, t0, proxy_zbar0(x, R0, t0, d0))
    return np.einsum("...ij,...j->...i", M, transform(x, Rp, tp, dd))


def proxy_phi_update_form(x, R0, t0, d0, dp):
    """phi(x; dp) ~= <R0^T ((1/d') R' x~ + dt)> (eq:phi_update), which drops
    the factor z0bar [ (1/d') R' x~ + t' ]_z^{-1} ~= 1."""
    Rp, tp, dd = _incremented(R0, t0, d0, dp)
    inner = np.einsum("...ij,...j->...i", Rp, homog(x)) / dd[..., None] + (tp - t0)
    return project(np.einsum("...ji,...j->...i", R0, inner))


def proxy_dphi(x, R0, t0, d0):
    """d phi / d dp at dp = 0, a 2x7 matrix per point (Sec. 3.4).

    phi = <phi*> with phi*(x; 0) = z0bar x~, so the quotient rule gives
    (1/z0bar) [[1, 0, -x], [0, 1, -y]] D*, where
    D* = d phi*/d dp = [ -M [R0 x~]_x | d0 M | M t0 ]."""
    x = np.asarray(x, float)
    zb = proxy_zbar0(x, R0, t0, d0)
    M = proxy_M(R0, t0, zb)
    Rx = np.einsum("...ij,...j->...i", R0, homog(x))
    Dw = -M @ skew(Rx)
    Dt = np.asarray(d0, float)[..., None, None] * M
    Dd = np.einsum("...ij,...j->...i", M, t0)[..., None]
    Dstar = np.concatenate([Dw, Dt, Dd], -1)  # [..., 3, 7]
    P = np.zeros(x.shape[:-1] + (2, 3))
    P[..., 0, 0] = 1.0
    P[..., 1, 1] = 1.0
    P[..., 0, 2] = -x[..., 0]
    P[..., 1, 2] = -x[..., 1]
    return (P @ Dstar) / zb[..., None, None]


def warp_dW(x, R, t, d):
    """d W(x; dp boxplus p) / d dp at dp = 0 for the forward-compositional
    increment (R' = exp(dw) R, t' = t + dt, d' = d + dd), 2x7 per point:
    d<v>/dv (1/v_z)[[1,0,-u_x],[0,1,-u_y]] times dv/dp = [-[R x~]_x | d I | t]."""
    v = transform(x, R, t, d)
    u = v[..., :2] / v[..., 2:3]
    P = np.zeros(v.shape[:-1] + (2, 3))
    P[..., 0, 0] = 1.0
    P[..., 1, 1] = 1.0
    P[..., 0, 2] = -u[..., 0]
    P[..., 1, 2] = -u[..., 1]
    P = P / v[..., 2, None, None]
    Rx = np.einsum("...ij,...j->...i", R, homog(x))
    dv = np.concatenate([-skew(Rx), np.asarray(d, float)[..., None, None] * np.eye(3),
                         np.broadcast_to(t[..., :, None], v.shape[:-1] + (3, 1))], -1)
    return P @ dv


def ordinary_ic_dW(x, d):
    """d W / d p at the identity warp R = I, t = 0 (Sec. 3.1), the Jacobian an
    ordinary IC formulation would use. Its depth column is t0 = 0."""
    x = np.asarray(x, float)
    I = np.broadcast_to(np.eye(3), x.shape[:-1] + (3, 3))
    return warp_dW(x, I, np.zeros(x.shape[:-1] + (3,)), np.asarray(d, float))


def ic_update(Rk, tk, dk, R0abs, d0, dw, dt, dd):
    """IC parameter update (Sec. 3.6, final equations):
        R_{k+1} = R_k R0^T dR^T R0,   t_{k+1} = t_k - R_k R0^T dt,
        d_{k+1} = d_k (d0 - dd) / d0.
    Applied per absolute frame with that frame's own rotation at p(0) (the
    paper has one template at the origin; with several hosts every frame keeps
    its own R0)."""
    dR = so3_exp(dw)
    R0T = np.swapaxes(R0abs, -1, -2)
    Rn = Rk @ R0T @ np.swapaxes(dR, -1, -2) @ R0abs
    tn = tk - np.einsum("...ij,...j->...i", Rk @ R0T, dt)
    dn = dk * (d0 - dd) / d0
    return Rn, tn, dn


def abs_maps(R_fh, t_h):
    """Constant 6x6 maps from absolute left increments of target f and host h
    to the left increment of their relative pose (R_fh = R_f R_h^T,
    t_fh = t_f - R_fh t_h), to first order:
        dtheta_rel = A dtheta_f + B dtheta_h,
        A = [[I, 0], [[R_fh t_h]_x, I]],
        B = [[-R_fh, 0], [-R_fh [t_h]_x, -R_fh]].
    With the host at the origin (t_h = 0, R_h = I) A is the identity and the
    paper's relative pose is the absolute one."""
    n = R_fh.shape[:-2]
    A = np.zeros(n + (6, 6))
    B = np.zeros(n + (6, 6))
    A[..., :3, :3] = np.eye(3)
    A[..., 3:, 3:] = np.eye(3)
    A[..., 3:, :3] = skew(np.einsum("...ij,...j->...i", R_fh, t_h))
    B[..., :3, :3] = -R_fh
    B[..., 3:, 3:] = -R_fh
    B[..., 3:, :3] = -R_fh @ skew(t_h)
    return A, B
