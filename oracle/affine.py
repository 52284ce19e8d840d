"""Photometric affine brightness per frame in the FC Gauss-Newton iteration
(oracle, FP64, test infrastructure).

The paper's prior-art discussion (Sec. 2) notes that direct methods have to
model the photometric response explicitly, as DSO does; the method itself
assumes brightness constancy. Reading used here (the paper gives no model):
every frame f has a log-gain a_f and an offset b_f, with I_f = e^{a_f} L + b_f
for a common radiance L. The target intensity is brought into the host
frame's photometric units before it is compared with the template:

    r = I_h(x) - b_h - g (I_f(W(x; p)) - b_f),    g = e^{a_h - a_f}.

At a = b = 0 this is the paper's residual. Its derivatives are the FC
Jacobian of the plain residual scaled by g for the geometry, and
    dr/da_h = -g (I_f - b_f),  dr/db_h = -1,  dr/da_f = g (I_f - b_f),  dr/db_f = g.
The unknowns are the poses (6 per frame), the brightness pairs (2 per frame)
and the inverse depths. The pinned frame keeps its pose and its (a, b) (its
rows become the identity with a zero right-hand side); the pose block, the
brightness block and the depths are each damped by damping_rel times the
mean of their diagonal, as in solver.py; the depths are eliminated by a Schur
complement and the rest solved by Cholesky; the brightness update is
additive. Everything else (frozen residual set per level, Huber weights,
convergence measure) is the FC iteration of gn.py.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import geometry as G
from . import residuals as RS
from . import solver as SV


def affine_residuals(prob, layout, poses, d, ab):
    """r of the model above, the valid mask, the target pixel q, the sampled
    target intensity I_f(q) and the gain g, per residual."""
    r_plain, valid, q, v = RS.warp_residuals(prob, layout, poses, d)
    If = layout.I0 - r_plain
    ah, bh = ab[layout.res_host, 0], ab[layout.res_host, 1]
    af, bf = ab[layout.res_target, 0], ab[layout.res_target, 1]
    g = np.exp(ah - af)
    r = layout.I0 - bh - g * (If - bf)
    return r, valid, q, If, g


def affine_jacobian(prob, layout, poses, d, ab, q, If, g):
    """Rows d r / d (relative pose increment, inverse depth) [R, 7] and
    d r / d (a_h, b_h, a_f, b_f) [R, 4]."""
    Jg = g[:, None] * RS.fc_jacobian(prob, layout, poses, d, q)
    bf = ab[layout.res_target, 1]
    e = g * (If - bf)
    Jp = np.stack([-e, -np.ones_like(e), e, g], -1)
    return Jg, Jp


def absolute_jacobian(layout, Jg, Jp, A_pair, B_pair, n_frames, n_points):
    """Sparse J on [pose_0 .. pose_{F-1}, (a, b)_0 .. (a, b)_{F-1}, d_0 .. d_{N-1}]."""
    R = Jg.shape[0]
    Jpose = Jg[:, :6]
    Jf = np.einsum("ri,rij->rj", Jpose, A_pair[layout.res_pair])
    Jh = np.einsum("ri,rij->rj", Jpose, B_pair[layout.res_pair])
    F6 = 6 * n_frames
    rows = np.repeat(np.arange(R), 17)
    cols = np.concatenate([
        6 * layout.res_target[:, None] + np.arange(6),
        6 * layout.res_host[:, None] + np.arange(6),
        (F6 + 2 * layout.res_host)[:, None] + np.arange(2),
        (F6 + 2 * layout.res_target)[:, None] + np.arange(2),
        (8 * n_frames + layout.res_point)[:, None],
    ], 1).reshape(-1)
    vals = np.concatenate([Jf, Jh, Jp, Jg[:, 6:7]], 1).reshape(-1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(R, 8 * n_frames + n_points))


class AffineFC:
    """FC Gauss-Newton over poses, per-frame affine brightness and inverse depths."""

    def __init__(self, prob, ab=None):
        self.prob = prob
        F = prob.n_frames
        self.poses = prob.poses_init.copy()
        self.d = prob.inv_depth_init.copy()
        self.ab = np.zeros((F, 2)) if ab is None else np.asarray(ab, float).copy()
        self.obs_live = np.ones(len(prob.obs_frame), bool)   # observations still in the window
        self.level = None
        self.history = []

    def start_level(self, level):
        P = self.prob
        self.level = level
        self.L = P.layout(level)
        _, valid0, _, _, _ = affine_residuals(P, self.L, self.poses, self.d, self.ab)
        self.frozen = valid0 & self.obs_live[self.L.res_obs]

    def drop_frame(self, f):
        """Keyframe drop (sliding window, Sec. 4.2), as in the plain iteration:
        every observation of a point hosted by f and every observation with
        target f leave the window; from the next step the frozen residual set
        and the convergence measure skip them."""
        P = self.prob
        assert 0 <= f < P.n_frames and f != P.pinned_frame, "the gauge frame cannot be dropped"
        obs_host = np.repeat(P.host_frame, np.diff(P.obs_ptr))
        self.obs_live &= ~((obs_host == f) | (P.obs_frame == f))
        if self.level is not None:
            self.frozen &= self.obs_live[self.L.res_obs]

    def step(self):
        P, L = self.prob, self.L
        F, N = P.n_frames, P.n_points
        r, valid, q, If, g = affine_residuals(P, L, self.poses, self.d, self.ab)
        act = self.frozen & valid
        r = np.where(act, r, 0.0)
        w = RS.huber_weight(r, P.huber_k) * act
        n_act = int(act.sum())
        st = {"level": self.level, "energy": float(np.sum(RS.huber_rho(r, P.huber_k) * act)),
              "sq": float(np.sum(r * r)), "n_active": n_act, "rmse": float(np.sqrt(np.sum(r * r) / max(n_act, 1)))}
        Jg, Jp = affine_jacobian(P, L, self.poses, self.d, self.ab, q, If, g)
        Jg[~act] = 0.0
        Jp[~act] = 0.0
        A, B = SV.pair_maps(L, self.poses)
        J = absolute_jacobian(L, Jg, Jp, A, B, F, N)
        H, gr = SV.normal_equations(J, w, r)
        n8, F6 = 8 * F, 6 * F
        Hxx = H[:n8, :n8].toarray()
        Hxd = H[:n8, n8:].tocsr()
        Hdd = H[n8:, n8:].diagonal().copy()
        dg = np.diag(Hxx).copy()
        mu_p = SV.damping_value(P.damping_rel, dg[:F6])
        mu_a = SV.damping_value(P.damping_rel, dg[F6:])
        mu_d = SV.damping_value(P.damping_rel, Hdd)
        Hxx[np.arange(F6), np.arange(F6)] += mu_p
        Hxx[np.arange(F6, n8), np.arange(F6, n8)] += mu_a
        Hdd = Hdd + mu_d
        S = Hxx - (Hxd @ sp.diags(1.0 / Hdd) @ Hxd.T).toarray()
        b = gr[:n8] - Hxd @ (gr[n8:] / Hdd)
        pin = []
        if P.pinned_frame >= 0:
            p = P.pinned_frame
            pin = list(range(6 * p, 6 * p + 6)) + [F6 + 2 * p, F6 + 2 * p + 1]
            S[pin, :] = 0.0
            S[:, pin] = 0.0
            S[pin, pin] = 1.0
            b[pin] = 0.0
        dx = -sla.cho_solve(sla.cho_factor(S, lower=True), b)
        dd = -(gr[n8:] + Hxd.T @ dx) / Hdd
        self.last = dict(S=S, b=b, Hdd=Hdd, r=r, w=w, act=act, mu=(mu_p, mu_a, mu_d))
        before_p, before_d = self.poses.copy(), self.d.copy()
        R, t = G.unpack(self.poses)
        d6 = dx[:F6].reshape(-1, 6)
        Rn, tn = G.boxplus_pose(R, t, d6[:, :3], d6[:, 3:])
        self.poses = G.pack(Rn, tn)
        self.ab = self.ab + dx[F6:].reshape(-1, 2)
        self.d = self.d + dd
        st["max_disp_px"] = RS.max_centre_displacement(L, before_p, before_d, self.poses, self.d, self.obs_live)
        st["step_pose"] = float(np.max(np.abs(dx[:F6]))) if F6 else 0.0
        st["step_brightness"] = float(np.max(np.abs(dx[F6:]))) if F else 0.0
        st["step_depth"] = float(np.max(np.abs(dd))) if dd.size else 0.0
        self.history.append(st)
        return st

    def iterate(self, level, n_iters):
        if self.level != level:
            self.start_level(level)
        return [self.step() for _ in range(n_iters)]

    def solve(self, max_iters_per_level, conv_px=5e-3):
        iters = []
        for level in reversed(range(self.prob.n_levels)):
            self.start_level(level)
            k = 0
            for k in range(1, max_iters_per_level + 1):
                if self.step()["max_disp_px"] < conv_px:
                    break
            iters.append(k)
        return iters

