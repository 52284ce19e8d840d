"""Ray-cast renderer for the synthetic scenes (input generation only).

Rays go through integer pixel centres of a pinhole camera; the image value is
the value-noise texture at the first surface hit, 0.5 on the background. No
lighting term is applied, so brightness constancy holds exactly up to the
optional additive image noise. The camera-frame depth Z of every hit is
returned as the ground-truth depth map.
"""
import numpy as np

from .noise import ValueNoise3

BACKGROUND = 0.5


class Sphere:
    def __init__(self, center, radius, seed, freq=4.0):
        self.c = np.asarray(center, float)
        self.r = float(radius)
        self.tex = ValueNoise3(seed)
        self.freq = freq

    def intersect(self, C, D):
        oc = C - self.c
        a = np.einsum("ij,ij->i", D, D)
        b = D @ oc
        cc = oc @ oc - self.r * self.r
        disc = b * b - a * cc
        s = np.full(D.shape[0], np.inf)
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        s0 = (-b - sq) / a
        s1 = (-b + sq) / a
        s = np.where(ok & (s0 > 1e-9), s0, np.where(ok & (s1 > 1e-9), s1, np.inf))
        return s


class Ellipsoid:
    def __init__(self, center, axes, seed, freq=4.0):
        self.c = np.asarray(center, float)
        self.ax = np.asarray(axes, float)
        self.tex = ValueNoise3(seed)
        self.freq = freq

    def intersect(self, C, D):
        Cp = (C - self.c) / self.ax
        Dp = D / self.ax
        a = np.einsum("ij,ij->i", Dp, Dp)
        b = Dp @ Cp
        cc = Cp @ Cp - 1.0
        disc = b * b - a * cc
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        s0 = (-b - sq) / a
        s1 = (-b + sq) / a
        return np.where(ok & (s0 > 1e-9), s0, np.where(ok & (s1 > 1e-9), s1, np.inf))


class Plane:
    """Finite rectangle: centre p0, unit normal n, in-plane axes e1/e2 with half sizes."""

    def __init__(self, p0, normal, e1, half1, half2, seed, freq=4.0):
        self.p0 = np.asarray(p0, float)
        self.n = np.asarray(normal, float) / np.linalg.norm(normal)
        e1 = np.asarray(e1, float)
        e1 = e1 - (e1 @ self.n) * self.n
        self.e1 = e1 / np.linalg.norm(e1)
        self.e2 = np.cross(self.n, self.e1)
        self.h1, self.h2 = float(half1), float(half2)
        self.tex = ValueNoise3(seed)
        self.freq = freq

    def intersect(self, C, D):
        dn = D @ self.n
        with np.errstate(divide="ignore", invalid="ignore"):
            s = ((self.p0 - C) @ self.n) / dn
        P = C[None, :] + s[:, None] * D
        rel = P - self.p0
        inside = (np.abs(rel @ self.e1) <= self.h1) & (np.abs(rel @ self.e2) <= self.h2)
        ok = np.isfinite(s) & (s > 1e-9) & inside
        return np.where(ok, s, np.inf)


class Box:
    """Axis-aligned box (in world axes) given by centre and half extents."""

    def __init__(self, center, half, seed, freq=4.0):
        self.c = np.asarray(center, float)
        self.h = np.asarray(half, float)
        self.tex = ValueNoise3(seed)
        self.freq = freq

    def intersect(self, C, D):
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / D
            t0 = (self.c - self.h - C) * inv
            t1 = (self.c + self.h - C) * inv
        tmin = np.nanmax(np.minimum(t0, t1), axis=1)
        tmax = np.nanmin(np.maximum(t0, t1), axis=1)
        ok = (tmax >= tmin) & (tmax > 1e-9)
        s = np.where(tmin > 1e-9, tmin, tmax)
        return np.where(ok, s, np.inf)


class Torus:
    """Torus around the world y axis through `center` (major R, minor r)."""

    def __init__(self, center, R, r, seed, freq=4.0):
        self.c = np.asarray(center, float)
        self.R, self.r = float(R), float(r)
        self.tex = ValueNoise3(seed)
        self.freq = freq
        self.bound = Sphere(center, R + r + 1e-3, 0)

    def _sdf(self, p):
        q = np.sqrt(p[:, 0] ** 2 + p[:, 2] ** 2) - self.R
        return np.sqrt(q * q + p[:, 1] ** 2) - self.r

    def intersect(self, C, D):
        n = D.shape[0]
        s_out = np.full(n, np.inf)
        # entry into the bounding sphere, then sphere tracing along the ray
        oc = C - self.c
        a = np.einsum("ij,ij->i", D, D)
        b = D @ oc
        cc = oc @ oc - self.bound.r ** 2
        disc = b * b - a * cc
        idx = np.nonzero(disc >= 0)[0]
        if idx.size == 0:
            return s_out
        sq = np.sqrt(disc[idx])
        s = np.maximum((-b[idx] - sq) / a[idx], 0.0)
        s_far = (-b[idx] + sq) / a[idx]
        Dn = D[idx] / np.sqrt(a[idx])[:, None]
        scale = np.sqrt(a[idx])
        alive = np.ones(idx.size, bool)
        hit = np.zeros(idx.size, bool)
        for _ in range(256):
            live = np.nonzero(alive)[0]
            if live.size == 0:
                break
            p = oc + s[live, None] * D[idx[live]]
            dist = self._sdf(p)
            done = dist < 1e-7
            hit[live[done]] = True
            alive[live[done]] = False
            s[live] = s[live] + np.where(done, 0.0, dist / scale[live])
            gone = s[live] > s_far[live]
            alive[live[gone]] = False
        s_out[idx[hit]] = s[hit]
        del Dn
        return s_out


def look_at(center, target, up=(0.0, 1.0, 0.0)):
    """World->camera (R, t) for a camera at `center` looking at `target`
    (camera x right, y down, z forward)."""
    C = np.asarray(center, float)
    z = np.asarray(target, float) - C
    z /= np.linalg.norm(z)
    u = np.asarray(up, float)
    y = -(u - (u @ z) * z)
    y /= np.linalg.norm(y)
    x = np.cross(y, z)
    R = np.stack([x, y, z])
    return R, -R @ C


def render(objects, R, t, K, width, height):
    """Returns (image float32 [H][W], depth float64 [H][W]; inf = background)."""
    fx, fy, cx, cy = K
    vv, uu = np.mgrid[0:height, 0:width].astype(float)
    dc = np.stack([(uu - cx) / fx, (vv - cy) / fy, np.ones_like(uu)], axis=-1).reshape(-1, 3)
    D = dc @ R  # rows: R^T dc
    C = -R.T @ t
    best = np.full(D.shape[0], np.inf)
    which = np.full(D.shape[0], -1)
    for k, ob in enumerate(objects):
        s = ob.intersect(C, D)
        closer = s < best
        best = np.where(closer, s, best)
        which = np.where(closer, k, which)
    img = np.full(D.shape[0], BACKGROUND)
    for k, ob in enumerate(objects):
        sel = np.nonzero(which == k)[0]
        if sel.size == 0:
            continue
        P = C[None, :] + best[sel, None] * D[sel]
        img[sel] = ob.tex.fractal(P - getattr(ob, "c", getattr(ob, "p0", 0.0)), base_freq=ob.freq)
    return img.reshape(height, width).astype(np.float32), best.reshape(height, width)
