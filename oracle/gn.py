"""Forward-compositional and proxy-template inverse-compositional Gauss-Newton
(oracle, FP64, test infrastructure).

FC (the paper's baseline, Sec. 1 and Sec. 2): at every iteration the Jacobian
of the residuals at the current parameters is formed, H = J^T W J is built and
factorized, and p <- dp boxplus p.

IC with proxy templates (Sec. 3.5): at the start of a pyramid level the
parameters are frozen as p(0); J (Sec. 3.4), the initial Huber weights W0 and
H = J^T W0 J are computed once. Every iteration then
  1. recomputes the Huber weights W at the current residuals,
  2. forms g = J^T W r,
  3. solves dp = -H^{-1} g,
  4. composes the warp with the inverse proxy update (Sec. 3.6, final
     equations).

Readings (the paper is silent): residuals are frozen to those usable at the
level's p(0) (a residual that later leaves the image, or whose point moves
behind the camera, gets weight 0 for that iteration); p(0) is re-centred at
the start of every pyramid level; the convergence test (Sec. 4.1) takes the
largest level-0 pixel displacement of any observation's point centre.

Dropping a keyframe (sliding window, dynamic Hessian): in the DSO
integration of Sec. 4.2 every change of the keyframe set still cost a new
Hessian, and a dynamic one is named as the next speed-up. drop_frame(f)
takes frame f's observations out of the window (those it hosts and those in
which it is the target; the frame stays as an unconstrained block, the
points it hosts stay with no observation) and, mid-level, forms the IC
system again from the rows of J and the weights W0 kept at p(0) without
linearizing the remaining residuals again: the result equals the level
set-up of the reduced problem at the same p(0).

Proxy re-centring (hybrid schedule): the final update equations of Sec. 3.6
rest on approximations that hold while the parameters stay near p(0) (the
proxy depth taken as 1/d0 and d0/d taken as 1). With recentre_every = m > 0
the IC iteration re-centres after every m iterations of a level: p(0) becomes
the current parameters and the level's linearization (J, W0, H, S) is formed
again there, exactly as at the level's start. m = 0 is the paper's IC.
"""
import numpy as np

from . import geometry as G
from . import image as IM
from . import residuals as RS
from . import solver as SV


class Problem:
    def __init__(self, images, intrinsics, poses, host_frame, host_uv, inv_depth, obs_ptr, obs_frame,
                 pattern, n_levels=1, huber_k=9.0 / 255.0, damping_rel=1e-6, pinned_frame=0):
        self.images = np.asarray(images)
        self.n_frames = self.images.shape[0]
        self.intrinsics = np.asarray(intrinsics, float)
        self.poses_init = np.asarray(poses, float).copy()
        self.host_frame = np.asarray(host_frame, np.int64)
        self.host_uv = np.asarray(host_uv, float)
        self.inv_depth_init = np.asarray(inv_depth, float).copy()
        self.obs_ptr = np.asarray(obs_ptr, np.int64)
        self.obs_frame = np.asarray(obs_frame, np.int64)
        self.pattern = np.asarray(pattern, float)
        self.n_levels = int(n_levels)
        self.huber_k = float(huber_k)
        self.damping_rel = float(damping_rel)
        self.pinned_frame = int(pinned_frame)
        self.pyr = IM.pyramid(self.images, self.n_levels)
        self.grads = [IM.central_gradients(s) for s in self.pyr]
        self._layouts = {}

    @staticmethod
    def from_scene(scene, **kw):
        args = dict(n_levels=scene.n_levels, huber_k=scene.huber_k)
        args.update(kw)
        return Problem(scene.images, scene.intrinsics, scene.poses_init, scene.host_frame, scene.host_uv,
                       scene.inv_depth_init, scene.obs_ptr, scene.obs_frame, scene.pattern, **args)

    @property
    def n_points(self):
        return self.host_frame.shape[0]

    def layout(self, level):
        if level not in self._layouts:
            self._layouts[level] = RS.Layout(self, level)
        return self._layouts[level]


class GaussNewton:
    def __init__(self, prob, mode, recentre_every=0):
        assert mode in ("fc", "ic")
        assert recentre_every >= 0
        self.prob = prob
        self.mode = mode
        self.recentre_every = int(recentre_every) if mode == "ic" else 0
        self.since = 0   # iterations since the last linearization of the level
        self.poses = prob.poses_init.copy()
        self.d = prob.inv_depth_init.copy()
        self.level = None
        self.history = []
        # observations still in the window (drop_frame), in the problem's order
        self.obs_live = np.ones(prob.obs_frame.shape[0], bool)

    # ---- level start: p(0), frozen residual set, and (IC) the constant system
    def start_level(self, level):
        P = self.prob
        L = P.layout(level)
        self.level = level
        self.L = L
        self.since = 0
        self.poses0 = self.poses.copy()
        self.d0 = self.d.copy()
        r0, valid0, _, _ = RS.warp_residuals(P, L, self.poses0, self.d0)
        self.frozen = valid0 & self.obs_live[L.res_obs]
        if self.mode == "ic":
            self.J0 = RS.ic_jacobian(L, self.poses0, self.d0)
            self.w0 = RS.huber_weight(r0, P.huber_k)
            self.A0, self.B0 = SV.pair_maps(L, self.poses0)
            self._ic_system()

    def _ic_system(self):
        """H = J^T W0 J over the frozen residuals and its reduced system, from
        the rows of J and the weights kept at p(0)."""
        P, L = self.prob, self.L
        J = np.where(self.frozen[:, None], self.J0, 0.0)
        self.J_rel = J
        self.Jabs = SV.absolute_jacobian(L, J, self.A0, self.B0, P.n_frames, P.n_points)
        H, _ = SV.normal_equations(self.Jabs, np.where(self.frozen, self.w0, 0.0), np.zeros(self.frozen.shape))
        self.H = H
        self.red = SV.Reduced(H, P.n_frames, P.damping_rel, P.pinned_frame)

    def drop_frame(self, f):
        """Take frame f's observations out of the window: every observation
        of a point hosted by f and every observation with target f. Within a
        level the frozen residual set loses them and (IC) the system is formed
        again from the rows kept at p(0), without a new linearization."""
        P = self.prob
        assert 0 <= f < P.n_frames and f != P.pinned_frame, "the gauge frame cannot be dropped"
        counts = np.diff(P.obs_ptr)
        obs_host = np.repeat(P.host_frame, counts)
        self.obs_live &= ~((obs_host == f) | (P.obs_frame == f))
        if self.level is not None:
            self.frozen &= self.obs_live[self.L.res_obs]
            if self.mode == "ic":
                self._ic_system()

    # ---- one Gauss-Newton iteration at the current level
    def step(self):
        if self.recentre_every and self.since == self.recentre_every:
            self.start_level(self.level)   # proxy re-centring: p(0) <- current parameters
        self.since += 1
        P, L = self.prob, self.L
        r, valid, q, v = RS.warp_residuals(P, L, self.poses, self.d)
        act = self.frozen & valid
        r = np.where(act, r, 0.0)
        w = RS.huber_weight(r, P.huber_k) * act
        n_act = int(act.sum())
        st = {
            "level": self.level,
            "energy": float(np.sum(RS.huber_rho(r, P.huber_k) * act)),
            "sq": float(np.sum(r * r)),
            "n_active": n_act,
            "rmse": float(np.sqrt(np.sum(r * r) / max(n_act, 1))),
        }
        poses_before, d_before = self.poses.copy(), self.d.copy()
        if self.mode == "fc":
            J = RS.fc_jacobian(P, L, self.poses, self.d, q)
            J[~act] = 0.0
            A, B = SV.pair_maps(L, self.poses)
            Jabs = SV.absolute_jacobian(L, J, A, B, P.n_frames, P.n_points)
            H, g = SV.normal_equations(Jabs, w, r)
            red = SV.Reduced(H, P.n_frames, P.damping_rel, P.pinned_frame)
            dth, dd, b = red.solve(g)
            self.last = dict(J=J, H=H, g=g, S=red.S, b=b, Hdd=red.Hdd, r=r, w=w, act=act)
            R, t = G.unpack(self.poses)
            dth6 = dth.reshape(-1, 6)
            Rn, tn = G.boxplus_pose(R, t, dth6[:, :3], dth6[:, 3:])
            self.poses = G.pack(Rn, tn)
            self.d = self.d + dd
        else:
            g = self.Jabs.T @ (w * r)
            dth, dd, b = self.red.solve(g)
            self.last = dict(g=g, b=b, r=r, w=w, act=act, S=self.red.S, Hdd=self.red.Hdd)
            R, t = G.unpack(self.poses)
            R0, _ = G.unpack(self.poses0)
            dth6 = dth.reshape(-1, 6)
            Rn, tn, dn = G.ic_update(R, t, self.d, R0, self.d0, dth6[:, :3], dth6[:, 3:], dd)
            self.poses = G.pack(Rn, tn)
            self.d = dn
        st["max_disp_px"] = RS.max_centre_displacement(L, poses_before, d_before, self.poses, self.d,
                                                       live=self.obs_live)
        st["step_pose"] = float(np.max(np.abs(dth))) if dth.size else 0.0
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
                st = self.step()
                if st["max_disp_px"] < conv_px:
                    break
            iters.append(k)
        return iters

    def evaluate(self, level=0):
        """Energy and photometric RMSE at the current parameters over the
        residuals usable at those parameters (fresh mask)."""
        P = self.prob
        L = P.layout(level)
        r, valid, _, _ = RS.warp_residuals(P, L, self.poses, self.d)
        valid = valid & self.obs_live[L.res_obs]
        r = np.where(valid, r, 0.0)
        n = int(valid.sum())
        return {"energy": float(np.sum(RS.huber_rho(r, P.huber_k) * valid)), "sq": float(np.sum(r * r)),
                "n_active": n, "rmse": float(np.sqrt(np.sum(r * r) / max(n, 1)))}
