"""Test-side helpers: per-observation sums of oracle quantities, laid out like the
library's debug records, and parameter error measures. Aggregation only; all
arithmetic of the method comes from `oracle`."""
import numpy as np

from oracle import geometry as G
from oracle import residuals as RS

REC = 40


def obs_records(layout, J, w, r, act, huber_k):
    """Per-observation sums of w J^T J (upper triangle), w J_th J_d, w J_d^2,
    w J r, Huber energy, r^2 and count, from oracle rows J (relative pose)."""
    O = layout.n_obs
    rec = np.zeros((O, REC))
    Jw = J * w[:, None]
    iu = np.triu_indices(6)
    outer = Jw[:, :6, None] * J[:, None, :6]
    cols = outer[:, iu[0], iu[1]]
    for k in range(21):
        rec[:, k] = np.bincount(layout.res_obs, cols[:, k], minlength=O)
    for k in range(6):
        rec[:, 21 + k] = np.bincount(layout.res_obs, Jw[:, k] * J[:, 6], minlength=O)
    rec[:, 27] = np.bincount(layout.res_obs, Jw[:, 6] * J[:, 6], minlength=O)
    for k in range(7):
        rec[:, 28 + k] = np.bincount(layout.res_obs, Jw[:, k] * r, minlength=O)
    rec[:, 35] = np.bincount(layout.res_obs, RS.huber_rho(r, huber_k) * act, minlength=O)
    rec[:, 36] = np.bincount(layout.res_obs, r * r * act, minlength=O)
    rec[:, 37] = np.bincount(layout.res_obs, act.astype(float), minlength=O)
    return rec


def rot_err(P1, P2):
    """Per-frame rotation difference (rad) of two pose arrays [F][12]."""
    R1, _ = G.unpack(P1)
    R2, _ = G.unpack(P2)
    # ||R1 - R2||_F = 2 sqrt(2) sin(theta / 2) for rotations: accurate near zero,
    # unlike the arccos of the trace
    d = np.linalg.norm((R1 - R2).reshape(len(R1), -1), axis=1)
    return 2.0 * np.arcsin(np.clip(d / (2.0 * np.sqrt(2.0)), 0.0, 1.0))


def trans_rel_err(P1, P2):
    t1, t2 = P1[:, 9:], P2[:, 9:]
    scale = max(np.linalg.norm(t2, axis=1).max(), 1e-12)
    return np.linalg.norm(t1 - t2, axis=1) / scale


def depth_errors_ok(d, d_ref, bar=1e-5):
    """Relative inverse-depth agreement of a result with the FP64 oracle,
    gated on the worst point (the measurement contract's 1e-5 relative bar).
    Returns (ok, 99th percentile, maximum); the statistics go into the
    assertion message."""
    rel = np.abs(d / d_ref - 1.0)
    worst = float(rel.max()) if rel.size else 0.0
    return worst <= bar, float(np.quantile(rel, 0.99)) if rel.size else 0.0, worst
