"""Normal equations and their solution (oracle, FP64, test infrastructure).

The Gauss-Newton step of Sec. 3.5 is dp = -H^{-1} g with H = J^T W J and
g = J^T W r. The oracle forms J on the absolute parameters as a sparse matrix
(one row per residual: 6 columns for the target frame, 6 for the host frame,
1 for the point's inverse depth) and applies the textbook formulas.

The paper assumes H invertible; it is not (the scale of the scene and, with
several hosts, the world frame are free). Reading used: the pose rows/columns
of one frame are replaced by the identity with a zero right-hand side, and
both diagonal blocks are damped by damping_rel times the mean of their
diagonal (computed before the pin; damping_rel itself when that mean is 0). The depths are eliminated by a Schur
complement; the reduced pose system is solved by Cholesky.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import geometry as G


def absolute_jacobian(layout, J_rel, A_pair, B_pair, n_frames, n_points):
    """Sparse J on [pose_0 .. pose_{F-1}, d_0 .. d_{N-1}] from relative rows:
    the target columns are J_rel A, the host columns J_rel B."""
    R = J_rel.shape[0]
    Jp = J_rel[:, :6]
    Jf = np.einsum("ri,rij->rj", Jp, A_pair[layout.res_pair])
    Jh = np.einsum("ri,rij->rj", Jp, B_pair[layout.res_pair])
    rows = np.repeat(np.arange(R), 13)
    cols = np.concatenate([
        6 * layout.res_target[:, None] + np.arange(6),
        6 * layout.res_host[:, None] + np.arange(6),
        (6 * n_frames + layout.res_point)[:, None],
    ], 1).reshape(-1)
    vals = np.concatenate([Jf, Jh, J_rel[:, 6:7]], 1).reshape(-1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(R, 6 * n_frames + n_points))


def normal_equations(J, w, r):
    """H = J^T W J, g = J^T W r (Sec. 3.5)."""
    Wd = sp.diags(w)
    H = (J.T @ Wd @ J).tocsr()
    g = J.T @ (w * r)
    return H, np.asarray(g).reshape(-1)


def damping_value(damping_rel, diag):
    """damping_rel times the mean of a block's diagonal; a block whose diagonal
    is all zero (nothing observed) is damped by damping_rel itself."""
    m = float(np.mean(diag)) if diag.size else 0.0
    return damping_rel * m if m > 0.0 else damping_rel


class Reduced:
    """Damped, pinned system split into pose and depth parts, its Schur
    complement S = Hpp - Hpd Hdd^{-1} Hdp and Cholesky factor."""

    def __init__(self, H, n_frames, damping_rel, pinned_frame):
        n6 = 6 * n_frames
        Hpp = H[:n6, :n6].toarray()
        self.Hpd = H[:n6, n6:].tocsr()
        Hdd = H[n6:, n6:].diagonal().copy()
        self.mu_p = damping_value(damping_rel, np.diag(Hpp))
        self.mu_d = damping_value(damping_rel, Hdd)
        Hpp = Hpp + self.mu_p * np.eye(n6)
        self.Hdd = Hdd + self.mu_d
        self.Hpp = Hpp
        S = Hpp - (self.Hpd @ sp.diags(1.0 / self.Hdd) @ self.Hpd.T).toarray()
        self.pin = slice(6 * pinned_frame, 6 * pinned_frame + 6) if pinned_frame >= 0 else None
        if self.pin is not None:
            S[self.pin, :] = 0.0
            S[:, self.pin] = 0.0
            S[self.pin, self.pin] = np.eye(6)
        self.S = S
        self.factor = sla.cho_factor(S, lower=True)
        self.n6 = n6

    def rhs(self, g):
        gp, gd = g[: self.n6], g[self.n6:]
        b = gp - self.Hpd @ (gd / self.Hdd)
        if self.pin is not None:
            b[self.pin] = 0.0
        return b

    def solve(self, g):
        """dp = -H^{-1} g through the Schur complement; returns (dtheta [6F], dd [N], b)."""
        b = self.rhs(g)
        dth = -sla.cho_solve(self.factor, b)
        gd = g[self.n6:]
        dd = -(gd + self.Hpd.T @ dth) / self.Hdd
        return dth, dd, b


def dense_solve(H, g, n_frames, damping_rel, pinned_frame):
    """The same step from the full (6F+N)^2 system without Schur elimination
    (used to check the Schur path on small problems)."""
    n6 = 6 * n_frames
    Hd = H.toarray() if sp.issparse(H) else np.array(H)
    mu_p = damping_value(damping_rel, np.diag(Hd)[:n6])
    mu_d = damping_value(damping_rel, np.diag(Hd)[n6:])
    Hd[np.arange(n6), np.arange(n6)] += mu_p
    Hd[np.arange(n6, Hd.shape[0]), np.arange(n6, Hd.shape[0])] += mu_d
    g = g.copy()
    if pinned_frame >= 0:
        s = slice(6 * pinned_frame, 6 * pinned_frame + 6)
        Hd[s, :] = 0.0
        Hd[:, s] = 0.0
        Hd[s, s] = np.eye(6)
        g[s] = 0.0
    step = -np.linalg.solve(Hd, g)
    return step[:n6], step[n6:]


def pair_maps(layout, poses):
    """A, B maps (geometry.abs_maps) of every pair at the given parameters."""
    R, t = G.unpack(poses)
    Rfh, _ = G.relative_pose(R[layout.pair_target], t[layout.pair_target], R[layout.pair_host], t[layout.pair_host])
    return G.abs_maps(Rfh, t[layout.pair_host])
