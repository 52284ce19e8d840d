"""Seeded synthetic photometric-BA problems.

Each builder returns a `Scene`: rendered frames, intrinsics, ground-truth and
perturbed poses (world = frame 0, world->camera), selected points with their
host pixel, ground-truth and perturbed inverse depth, and the CSR list of the
frames that observe each point. The five workloads follow the problem sizes
used for the measurements: tiny sphere, mid ellipsoid, precision torus,
batched windows of planes and spheres, and the large multi-object scene.
Nothing here evaluates the photometric objective or its derivatives.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from .render import Box, Ellipsoid, Plane, Sphere, Torus, look_at, render

# 8-pixel patch pattern (du, dv) in level-l pixels: a diamond of radius 2
# around the point centre.
PATTERN8 = np.array(
    [[0, 0], [0, -2], [-1, -1], [1, -1], [-2, 0], [2, 0], [-1, 1], [1, 1]], dtype=np.int32
)
HUBER_K = 9.0 / 255.0


@dataclass
class Scene:
    name: str
    images: np.ndarray  # float32 [F][H][W]
    intrinsics: np.ndarray  # float64 [F][4] fx fy cx cy (level 0)
    poses_gt: np.ndarray  # float64 [F][12] world->camera, R row-major then t
    poses_init: np.ndarray  # float64 [F][12]
    host_frame: np.ndarray  # int32 [N]
    host_uv: np.ndarray  # float32 [N][2] level-0 pixel (integers)
    inv_depth_gt: np.ndarray  # float64 [N]
    inv_depth_init: np.ndarray  # float64 [N]
    obs_ptr: np.ndarray  # int32 [N+1]
    obs_frame: np.ndarray  # int32 [O]
    n_levels: int = 1
    huber_k: float = HUBER_K
    pattern: np.ndarray = field(default_factory=lambda: PATTERN8.copy())
    meta: dict = field(default_factory=dict)

    @property
    def n_frames(self):
        return self.images.shape[0]

    @property
    def height(self):
        return self.images.shape[1]

    @property
    def width(self):
        return self.images.shape[2]

    @property
    def n_points(self):
        return self.host_frame.shape[0]

    @property
    def n_obs(self):
        return int(self.obs_ptr[-1])

    def n_residuals(self):
        return self.n_obs * self.pattern.shape[0]

    def save(self, path):
        d = {k: getattr(self, k) for k in (
            "images", "intrinsics", "poses_gt", "poses_init", "host_frame", "host_uv",
            "inv_depth_gt", "inv_depth_init", "obs_ptr", "obs_frame", "pattern")}
        np.savez(path, name=self.name, n_levels=self.n_levels, huber_k=self.huber_k, **d)

    @staticmethod
    def load(path):
        z = np.load(path)
        kw = {k: z[k] for k in z.files if k not in ("name", "n_levels", "huber_k")}
        return Scene(name=str(z["name"]), n_levels=int(z["n_levels"]), huber_k=float(z["huber_k"]), **kw)


def _rot(axis, ang):
    """Rotation matrix about a unit axis (Rodrigues), for input perturbation only."""
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)


def _pack(R, t):
    return np.concatenate([R.reshape(9), t])


def _orbit(n, radius, height, start_deg, step_deg, target=(0.0, 0.0, 0.0)):
    poses = []
    for i in range(n):
        a = math.radians(start_deg + i * step_deg)
        C = np.array([radius * math.sin(a), -height, -radius * math.cos(a)])
        poses.append(look_at(C, target, up=(0.0, -1.0, 0.0)))
    return poses


def _to_frame0(poses):
    R0, t0 = poses[0]
    out = []
    for R, t in poses:
        Rr = R @ R0.T
        out.append((Rr, t - Rr @ t0))
    return out


def _select_points(img, depth, n_pts, margin, focal):
    """Top-n gradient-magnitude pixels whose 5x5 window lies on a surface.
    Pixels whose surface faces the camera are preferred: the fronto-parallel
    patch model of a point (one inverse depth for all its pattern pixels) is
    accurate there. Ties are broken by row-major index. Returns candidate
    (v, u) arrays in rank order."""
    H, W = img.shape
    gu = np.zeros_like(img, dtype=np.float64)
    gv = np.zeros_like(img, dtype=np.float64)
    gu[:, 1:-1] = 0.5 * (img[:, 2:].astype(np.float64) - img[:, :-2])
    gv[1:-1, :] = 0.5 * (img[2:, :].astype(np.float64) - img[:-2, :])
    mag = np.hypot(gu, gv)
    on = np.isfinite(depth)
    win = np.ones_like(on)
    for dv in range(-2, 3):
        for du in range(-2, 3):
            win &= np.roll(np.roll(on, -dv, 0), -du, 1)
    # slant of the surface: the slope of the depth map per pixel, times f/Z,
    # is the tangent of the angle between the surface and the image plane
    Zs = np.where(on, depth, 1.0)
    dzu = np.zeros_like(Zs)
    dzv = np.zeros_like(Zs)
    dzu[:, 1:-1] = 0.5 * (Zs[:, 2:] - Zs[:, :-2])
    dzv[1:-1, :] = 0.5 * (Zs[2:, :] - Zs[:-2, :])
    slant = np.hypot(dzu, dzv) * focal / Zs
    ok = win.copy()
    ok[:margin, :] = False
    ok[H - margin:, :] = False
    ok[:, :margin] = False
    ok[:, W - margin:] = False
    # tiers of slant (tan 19, 35, 45 degrees): a point is ranked first by the
    # lowest tier it belongs to, then by gradient magnitude
    tier = np.where(slant < 0.35, 0, np.where(slant < 0.7, 1, np.where(slant < 1.0, 2, 3)))
    ok &= tier < 3
    idx = np.nonzero(ok.reshape(-1))[0]
    order = np.lexsort((idx, -mag.reshape(-1)[idx], tier.reshape(-1)[idx]))
    sel = idx[order]
    return sel // W, sel % W


def _visible(Xw, R, t, K, depth, W, H, margin=6, tol=1e-2):
    Xc = Xw @ R.T + t
    Z = Xc[:, 2]
    good = Z > 1e-6
    Zs = np.where(good, Z, 1.0)
    u = K[0] * Xc[:, 0] / Zs + K[2]
    v = K[1] * Xc[:, 1] / Zs + K[3]
    good &= (u >= margin) & (u <= W - 1 - margin) & (v >= margin) & (v <= H - 1 - margin)
    ui = np.clip(np.rint(u), 0, W - 1).astype(int)
    vi = np.clip(np.rint(v), 0, H - 1).astype(int)
    dz = depth[vi, ui]
    good &= np.isfinite(dz) & (np.abs(dz - Z) < tol * Z)
    return good


def _build(name, objects, poses_scene, W, H, hosts, n_per_host, target_fn, n_levels, noise_sigma,
           seed, perturb="paper"):
    rng = np.random.default_rng(seed)
    f = 0.9375 * W
    K = np.array([f, f, (W - 1) / 2.0, (H - 1) / 2.0])
    F = len(poses_scene)
    imgs, depths = [], []
    for R, t in poses_scene:
        im, dp = render(objects, R, t, K, W, H)
        imgs.append(im)
        depths.append(dp)
    images = np.stack(imgs)
    if noise_sigma > 0:
        images = (images + rng.normal(0.0, noise_sigma, images.shape)).astype(np.float32)
    poses = _to_frame0(poses_scene)
    margin = 5 * 2 ** (n_levels - 1) + 2

    host_frame, host_uv, inv_d, obs_ptr, obs_frame = [], [], [], [0], []
    for h in hosts:
        vs, us = _select_points(images[h], depths[h], n_per_host, margin, f)
        Rh, th = poses[h]
        Z = depths[h][vs, us]
        xh = np.stack([(us - K[2]) / K[0], (vs - K[3]) / K[1], np.ones_like(Z, dtype=float)], 1) * Z[:, None]
        Xw = (xh - th) @ Rh
        base = len(host_frame)
        # candidate target frames per point (depends on the point's global index)
        cand = [target_fn(h, base + i) for i in range(min(len(vs), 64))]
        uniq_frames = sorted({fr for c in cand for fr in c} | set(
            fr for i in range(0, len(vs), max(1, len(vs) // 16)) for fr in target_fn(h, base + i)))
        vis = {fr: _visible(Xw, poses[fr][0], poses[fr][1], K, depths[fr], W, H) for fr in uniq_frames}
        kept = 0
        for i in range(len(vs)):
            n_glob = base + kept
            seen = []
            for fr in sorted(target_fn(h, n_glob)):
                if fr not in vis:
                    vis[fr] = _visible(Xw, poses[fr][0], poses[fr][1], K, depths[fr], W, H)
                if vis[fr][i]:
                    seen.append(fr)
            if not seen:
                continue
            host_frame.append(h)
            host_uv.append((us[i], vs[i]))
            inv_d.append(1.0 / Z[i])
            obs_frame.extend(seen)
            obs_ptr.append(len(obs_frame))
            kept += 1
            if kept == n_per_host:
                break
    poses_gt = np.stack([_pack(R, t) for R, t in poses])

    poses_init = poses_gt.copy()
    inv_d = np.asarray(inv_d, float)
    if perturb == "fixed":
        # 1 degree about a seeded uniform axis (left-multiplied), t += 1% |t|
        # along a seeded direction, inverse depth *= 1 + 5% N(0,1)
        for fr in range(1, F):
            axis = rng.normal(size=3)
            dirn = rng.normal(size=3)
            R = _rot(axis, math.radians(1.0)) @ poses_gt[fr, :9].reshape(3, 3)
            t = poses_gt[fr, 9:] + 0.01 * np.linalg.norm(poses_gt[fr, 9:]) * dirn / np.linalg.norm(dirn)
            poses_init[fr] = _pack(R, t)
        inv_d_init = inv_d * (1.0 + 0.05 * rng.normal(size=inv_d.shape))
    else:
        # Gaussian noise of sigma = 1e-3 on every parameter in units where the
        # mean point depth is one (the protocol of the paper's Sec. 4.1):
        # rotation vector and translation/Zbar, and inverse depth * Zbar
        zbar = float(np.mean(1.0 / inv_d))
        for fr in range(1, F):
            w = 1e-3 * rng.normal(size=3)
            R = _rot(w, np.linalg.norm(w)) @ poses_gt[fr, :9].reshape(3, 3)
            t = poses_gt[fr, 9:] + 1e-3 * zbar * rng.normal(size=3)
            poses_init[fr] = _pack(R, t)
        inv_d_init = inv_d + (1e-3 / zbar) * rng.normal(size=inv_d.shape)
    # frame 0 (the world frame) is never perturbed
    return Scene(
        name=name,
        images=images.astype(np.float32),
        intrinsics=np.tile(K, (F, 1)),
        poses_gt=poses_gt,
        poses_init=poses_init,
        host_frame=np.asarray(host_frame, np.int32),
        host_uv=np.asarray(host_uv, np.float32).reshape(-1, 2),
        inv_depth_gt=inv_d,
        inv_depth_init=inv_d_init,
        obs_ptr=np.asarray(obs_ptr, np.int32),
        obs_frame=np.asarray(obs_frame, np.int32),
        n_levels=n_levels,
        meta={"seed": seed, "noise_sigma": noise_sigma, "hosts": list(hosts), "perturb": perturb},
    )


def tiny(seed=1, n_points=500, width=320, height=240):
    """Unit sphere, 4 cameras on a radius-3 arc 15 degrees apart, host frame 0,
    observations in frames 1-3 where visible; one pyramid level, no image noise;
    poses perturbed by 1 degree / 1% translation, inverse depths by 5%."""
    objs = [Sphere((0, 0, 0), 1.0, seed + 100, freq=2.0)]
    poses = _orbit(4, 3.0, 0.0, 0.0, 15.0)
    return _build("tiny", objs, poses, width, height, [0], n_points,
                  lambda h, n: [1, 2, 3], 1, 0.0, seed, perturb="fixed")


def mid(seed=2, n_per_host=4000, width=640, height=480, n_frames=30, reach=3, noise_sigma=2.0 / 255.0):
    """Ellipsoid (1.0/0.8/0.6), 30 cameras on a full orbit of radius 3, hosts
    0,6,12,18,24, targets the visible frames within +-reach (3: up to 36
    degrees from the host), 3 levels, image noise sigma noise_sigma (2/255)."""
    objs = [Ellipsoid((0, 0, 0), (1.0, 0.8, 0.6), seed + 100)]
    poses = _orbit(n_frames, 3.0, 0.8, 0.0, 360.0 / n_frames)
    hosts = list(range(0, n_frames - 5, 6))[:5]
    offsets = [k for k in range(-reach, reach + 1) if k != 0]

    def targets(h, n):
        return sorted({(h + k) % n_frames for k in offsets})

    return _build("mid", objs, poses, width, height, hosts, n_per_host, targets, 3, noise_sigma, seed)


def precision(seed=3, n_per_host=20000, width=640, height=480, n_frames=120):
    """Torus (R=1, r=0.4) seen from a 120-camera orbit of radius 3.5 at height
    1.5; 10 hosts (every 12th frame) x 20000 points; each point observes 4 of
    the 12 frames around its host, offsets {+-1,+-4}, {+-2,+-5} or {+-3,+-6}
    chosen by point index mod 3; 3 levels, noise 2/255."""
    objs = [Torus((0, 0, 0), 1.0, 0.4, seed + 100)]
    poses = _orbit(n_frames, 3.5, 1.5, 0.0, 360.0 / n_frames)
    hosts = list(range(0, n_frames, 12))[:10]
    sets = [(-4, -1, 1, 4), (-5, -2, 2, 5), (-6, -3, 3, 6)]

    def targets(h, n):
        return sorted({(h + k) % n_frames for k in sets[n % 3]})

    return _build("precision", objs, poses, width, height, hosts, n_per_host, targets, 3, 2.0 / 255.0, seed)


def learned(seed=5, n_per_host=30000, width=640, height=480, n_frames=300):
    """Three spheres and a box on a 300-camera orbit; 30 hosts (every 10th)
    x 30000 points, 4 targets per point interleaved over +-5 frames."""
    objs = [Sphere((-0.8, 0.0, 0.3), 0.5, seed + 100), Sphere((0.7, -0.2, 0.5), 0.45, seed + 101),
            Sphere((0.0, 0.3, -0.8), 0.55, seed + 102), Box((0.1, 0.45, 0.1), (0.35, 0.3, 0.35), seed + 103)]
    poses = _orbit(n_frames, 4.0, 1.2, 0.0, 360.0 / n_frames)
    hosts = list(range(0, n_frames, 10))[:30]
    sets = [(-3, -1, 1, 3), (-4, -2, 2, 4), (-5, -3, 3, 5), (-4, -1, 1, 4), (-5, -2, 2, 5)]

    def targets(h, n):
        return sorted({(h + k) % n_frames for k in sets[n % 5]})

    return _build("learned", objs, poses, width, height, hosts, n_per_host, targets, 3, 2.0 / 255.0, seed)


def window(seed, n_kf=None, pts_per_host=None, width=1280, height=720, n_levels=1):
    """One sliding window of the batched workload: a seeded arc of 5-9
    keyframes over textured planes and spheres; every keyframe hosts
    1000-3000 points; targets are the other keyframes where visible; one
    pyramid level by default (the windows run a fixed number of iterations from
    the small perturbation of the paper's protocol)."""
    rng = np.random.default_rng(10_000 + seed)
    n_kf = int(rng.integers(5, 10)) if n_kf is None else n_kf
    pts = int(rng.integers(1000, 3001)) if pts_per_host is None else pts_per_host
    objs = [Plane((0, 1.0, 0), (0, -1, 0), (1, 0, 0), 4.0, 4.0, seed * 7 + 1),
            Plane((0, 0, 2.5), (0, 0, -1), (1, 0, 0), 4.0, 3.0, seed * 7 + 2)]
    for k in range(3):
        c = (rng.uniform(-1.2, 1.2), rng.uniform(-0.2, 0.6), rng.uniform(-0.8, 1.2))
        objs.append(Sphere(c, rng.uniform(0.25, 0.5), seed * 7 + 3 + k))
    start = rng.uniform(-20.0, 0.0)
    poses = _orbit(n_kf, 4.0, 0.6, 180.0 + start, 3.0, target=(0.0, 0.2, 0.5))

    def targets(h, n):
        return [f for f in range(n_kf) if f != h]

    return _build(f"window{seed}", objs, poses, width, height, list(range(n_kf)), pts, targets, n_levels,
                  2.0 / 255.0, seed)


BUILDERS = {"tiny": tiny, "mid": mid, "precision": precision, "learned": learned}
