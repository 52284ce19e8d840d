"""Front end that produces the starting parameters p(0) (oracle, FP64 and exact
integers, test infrastructure).

Sec. 4.1 obtains its base solution in four steps: Harris corners, robust KLT
tracking of those corners, a geometric bundle adjustment with outlier removal
for the first poses and depths, then the forward-compositional photometric
bundle adjustment (the FC iteration of gn.py). The paper names the methods and
gives no parameters; the readings used here are:

Corners (Harris and Stephens)
  * the image is quantized to 8 bits, q = rint(float32(I) * 255) clamped to
    [0, 255] (camera images are 8-bit), so that everything after it is exact
    integer arithmetic and the corner set does not depend on rounding;
  * gradients are central differences times two, gx = q[v, u+1] - q[v, u-1],
    gy = q[v+1, u] - q[v-1, u];
  * the structure tensor sums gx^2, gy^2, gx gy over a 5 x 5 box window;
  * the response uses kappa = 1/16, scaled by 16 so that it stays an integer:
    R = 16 (Sxx Syy - Sxy^2) - (Sxx + Syy)^2;
  * a candidate lies at least `margin` pixels inside the image, has
    R > min_response and is a 3 x 3 local maximum (strictly larger than the
    neighbours before it in raster order, at least as large as those after);
  * one corner per cell of cell x cell pixels (the largest R, then the first in
    raster order), then the max_corners strongest cells (R descending, then
    raster order). The cells spread the corners over the image, as a "good
    features" detector does.

Tracking (Lucas and Kanade, translational, coarse to fine)
  * in its inverse-compositional form: the template is the window of
    (2 radius + 1)^2 pixels around the host position, bilinearly sampled, with
    the bilinear central-difference gradients of image.py; H = sum G G^T is
    formed once per level and every iteration takes d <- d - H^{-1} sum G e,
    e = I_target(x + d) - T(x);
  * it starts from a predicted position in the target (the caller's, e.g. from
    rough poses), runs a fixed number of iterations per level from the coarsest
    level to level 0 (the displacement doubles from one level to the next);
  * a track is lost when the template window leaves the usable area of
    image.py at some level, when the smaller eigenvalue of H divided by the
    window's pixel count is below min_eig (too little texture), or when an
    iteration's window leaves the usable area;
  * robustness: the position found is tracked back into the host the same way
    (starting from the host position); the track is kept if that returns
    within fb_px of where it started.

Geometric bundle adjustment
  * one 2-D residual per observation, e = pi_f(R x~ + d t) - z (level-0
    pixels, the relative pose and inverse-depth parameterization of eq:warp,
    z the tracked position); its Jacobian is diag(fx, fy) times the warp
    derivative of the FC increment (geometry.warp_dW);
  * Huber weight on |e| with threshold huber_px, shared by both rows; energy
    sum rho(|e|), squared error sum |e|^2;
  * the same normal equations, absolute-pose maps, gauge pin, damping, depth
    Schur complement and FC update as the photometric FC iteration; an
    observation whose point lies behind the target camera contributes nothing
    in that iteration;
  * the same convergence test (largest point-centre displacement, Sec. 4.1);
  * outlier removal: after the first solve, observations with |e| above
    outlier_px (or behind the camera) are removed and the solve runs again
    from where it stopped.
"""
import numpy as np

from . import geometry as G
from . import image as IM
from . import residuals as RS
from . import solver as SV

# ---------------------------------------------------------------- corners


def quantize8(img):
    """Level-0 image (float32 values) -> 8-bit integers: rint(I * 255) in
    single precision (half to even), clamped to [0, 255]."""
    q = np.rint(np.asarray(img, np.float32) * np.float32(255.0))
    return np.clip(q, 0, 255).astype(np.int64)


def harris_response(img):
    """Integer Harris response 16 det(S) - tr(S)^2 of every pixel whose 5 x 5
    window of central differences lies inside the image (rows and columns
    3 .. size - 4); other entries are 0 and never candidates."""
    q = quantize8(img)
    H, W = q.shape
    gx = np.zeros_like(q)
    gy = np.zeros_like(q)
    gx[:, 1:-1] = q[:, 2:] - q[:, :-2]
    gy[1:-1, :] = q[2:, :] - q[:-2, :]
    prods = (gx * gx, gy * gy, gx * gy)
    R = np.zeros((H, W), np.int64)
    if H < 7 or W < 7:
        return R
    sums = []
    for p in prods:
        s = np.zeros((H - 6, W - 6), np.int64)
        for di in range(-2, 3):
            for dj in range(-2, 3):
                s += p[3 + di: H - 3 + di, 3 + dj: W - 3 + dj]
        sums.append(s)
    sxx, syy, sxy = sums
    R[3: H - 3, 3: W - 3] = 16 * (sxx * syy - sxy * sxy) - (sxx + syy) ** 2
    return R


def local_maxima(R, margin, min_response):
    """Candidate mask: inside the margin, R > min_response, and a 3 x 3 local
    maximum with ties going to the first pixel in raster order."""
    H, W = R.shape
    m = max(int(margin), 4)
    cand = np.zeros((H, W), bool)
    if H - 2 * m <= 0 or W - 2 * m <= 0:
        return cand
    c = R[m: H - m, m: W - m]
    ok = c > min_response
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            nb = R[m + di: H - m + di, m + dj: W - m + dj]
            before = di < 0 or (di == 0 and dj < 0)
            ok &= (c > nb) if before else (c >= nb)
    cand[m: H - m, m: W - m] = ok
    return cand


def detect_corners(img, cell=8, margin=8, min_response=0, max_corners=2000):
    """Corners of one image: (uv [K, 2] int64 as (column, row), response [K]),
    strongest first (see the module docstring)."""
    R = harris_response(img)
    H, W = R.shape
    cand = local_maxima(R, margin, min_response)
    vi, ui = np.nonzero(cand)
    if vi.size == 0:
        return np.zeros((0, 2), np.int64), np.zeros(0, np.int64)
    resp = R[vi, ui]
    idx = vi * W + ui
    cell_id = (vi // cell) * ((W + cell - 1) // cell) + ui // cell
    # best of each cell: largest response, then smallest raster index
    order = np.lexsort((idx, -resp, cell_id))
    first = np.ones(order.size, bool)
    first[1:] = cell_id[order][1:] != cell_id[order][:-1]
    win = order[first]
    # strongest cells first, ties in raster order
    win = win[np.lexsort((idx[win], -resp[win]))][:max_corners]
    return np.stack([ui[win], vi[win]], -1).astype(np.int64), resp[win]


# ---------------------------------------------------------------- tracking

TRACK_OK, TRACK_LOW_TEXTURE, TRACK_LEFT_IMAGE, TRACK_FB = 0, 1, 2, 3


def _window(radius):
    r = np.arange(-radius, radius + 1, dtype=float)
    dv, du = np.meshgrid(r, r, indexing="ij")   # rows outer, columns inner
    return np.stack([du.reshape(-1), dv.reshape(-1)], -1)


def _lk_one_way(pyr, grads, src, xs, dst, guess, radius, n_iters, min_eig):
    """Coarse-to-fine translational LK of the window around xs (level-0 pixels)
    in frame src into frame dst, from the level-0 guess; returns (level-0
    positions [T, 2], status [T])."""
    L = len(pyr)
    T = xs.shape[0]
    off = _window(radius)
    npx = off.shape[0]
    d = (guess - xs) / 2.0 ** (L - 1)
    status = np.full(T, TRACK_OK)
    for l in reversed(range(L)):
        if l < L - 1:
            d = 2.0 * d
        stack = pyr[l]
        gu, gv = grads[l]
        Hh, Ww = stack.shape[1], stack.shape[2]
        xl = IM.level_pixel(xs, l)
        tp = xl[:, None, :] + off[None, :, :]
        inside = IM.in_bounds(tp[..., 0], tp[..., 1], Ww, Hh).all(1)
        fr = np.repeat(src[:, None], npx, 1)
        tmpl = IM.bilinear(stack, fr, tp[..., 0], tp[..., 1])
        gx = IM.bilinear(gu, fr, tp[..., 0], tp[..., 1])
        gy = IM.bilinear(gv, fr, tp[..., 0], tp[..., 1])
        a = np.sum(gx * gx, 1)
        b = np.sum(gx * gy, 1)
        c = np.sum(gy * gy, 1)
        lam = 0.5 * (a + c) - np.sqrt(0.25 * (a - c) ** 2 + b * b)
        status = np.where((status == TRACK_OK) & ~inside, TRACK_LEFT_IMAGE, status)
        status = np.where((status == TRACK_OK) & (lam / npx < min_eig), TRACK_LOW_TEXTURE, status)
        det = a * c - b * b
        frd = np.repeat(dst[:, None], npx, 1)
        for _ in range(n_iters):
            live = status == TRACK_OK
            if not live.any():
                break
            pos = xl[:, None, :] + d[:, None, :] + off[None, :, :]
            ok = IM.in_bounds(pos[..., 0], pos[..., 1], Ww, Hh).all(1)
            status = np.where(live & ~ok, TRACK_LEFT_IMAGE, status)
            live = status == TRACK_OK
            e = IM.bilinear(stack, frd, pos[..., 0], pos[..., 1]) - tmpl
            bx = np.sum(gx * e, 1)
            by = np.sum(gy * e, 1)
            dets = np.where(live, det, 1.0)
            step = np.stack([(c * bx - b * by) / dets, (a * by - b * bx) / dets], -1)
            d = np.where(live[:, None], d - step, d)
    return xs + d, status


def track(pyr, grads, host, host_uv, target, guess_uv, radius=4, n_iters=10, min_eig=1e-6, fb_px=0.5):
    """Robust tracks of host_uv [T, 2] (level-0 pixels in frames host [T]) into
    frames target [T] starting from guess_uv: (positions [T, 2], status [T],
    forward-backward distance [T]). pyr / grads: image.pyramid and
    image.central_gradients of each level."""
    host = np.asarray(host, np.int64)
    target = np.asarray(target, np.int64)
    xs = np.asarray(host_uv, float)
    fwd, st = _lk_one_way(pyr, grads, host, xs, target, np.asarray(guess_uv, float), radius, n_iters, min_eig)
    back, stb = _lk_one_way(pyr, grads, target, fwd, host, xs, radius, n_iters, min_eig)
    fb = np.hypot(back[:, 0] - xs[:, 0], back[:, 1] - xs[:, 1])
    status = np.where(st != TRACK_OK, st, np.where(stb != TRACK_OK, stb, TRACK_OK))
    status = np.where((status == TRACK_OK) & ~(fb <= fb_px), TRACK_FB, status)
    return fwd, status, fb


# ---------------------------------------------------------------- geometric BA


class _GeoLayout:
    """Index arrays of the observations (CSR order) and of their 2 rows each."""

    def __init__(self, n_frames, intrinsics, host_frame, host_uv, obs_ptr, obs_frame):
        N = host_frame.shape[0]
        counts = np.diff(obs_ptr)
        self.obs_point = np.repeat(np.arange(N), counts)
        self.obs_target = np.asarray(obs_frame, np.int64)
        self.obs_host = host_frame[self.obs_point]
        key = self.obs_host * n_frames + self.obs_target
        uniq, inv = np.unique(key, return_inverse=True)
        self.pair_host = uniq // n_frames
        self.pair_target = uniq % n_frames
        self.obs_pair = inv
        Kh = intrinsics[self.obs_host]
        c = host_uv[self.obs_point]
        self.obs_x0 = np.stack([(c[:, 0] - Kh[:, 2]) / Kh[:, 0], (c[:, 1] - Kh[:, 3]) / Kh[:, 1]], -1)
        self.obs_K0t = intrinsics[self.obs_target]
        # rows: 2 per observation (u then v)
        self.res_obs = np.repeat(np.arange(self.obs_point.size), 2)
        self.res_pair = self.obs_pair[self.res_obs]
        self.res_target = self.obs_target[self.res_obs]
        self.res_host = self.obs_host[self.res_obs]
        self.res_point = self.obs_point[self.res_obs]


class GeometricBA:
    """Reprojection-error bundle adjustment of poses and inverse depths (see the
    module docstring), FP64."""

    def __init__(self, intrinsics, poses, host_frame, host_uv, inv_depth, obs_ptr, obs_frame, obs_uv,
                 huber_px=2.0, damping_rel=1e-6, pinned_frame=0):
        self.K = np.asarray(intrinsics, float)
        self.poses = np.asarray(poses, float).copy()
        self.n_frames = self.poses.shape[0]
        self.host_frame = np.asarray(host_frame, np.int64)
        self.host_uv = np.asarray(host_uv, float)
        self.d = np.asarray(inv_depth, float).copy()
        self.z = np.asarray(obs_uv, float)
        self.huber_px = float(huber_px)
        self.damping_rel = float(damping_rel)
        self.pinned_frame = int(pinned_frame)
        self.L = _GeoLayout(self.n_frames, self.K, self.host_frame, self.host_uv, np.asarray(obs_ptr, np.int64),
                            obs_frame)
        self.inlier = np.ones(self.L.obs_point.size, bool)
        self.history = []

    def reprojection(self, poses=None, d=None):
        """e [O, 2] (level-0 pixels) and v_z > 0 of every observation."""
        poses = self.poses if poses is None else poses
        d = self.d if d is None else d
        q, ok = RS.centre_pixels(self.L, poses, d)
        return q - self.z, ok

    def _rows(self):
        """Residual rows, Huber weights, active rows and the relative Jacobian
        rows [2 O, 7] at the current parameters."""
        L = self.L
        R, t = G.unpack(self.poses)
        Rr, tr = G.relative_pose(R[L.pair_target], t[L.pair_target], R[L.pair_host], t[L.pair_host])
        Ro, to = Rr[L.obs_pair], tr[L.obs_pair]
        dW = G.warp_dW(L.obs_x0, Ro, to, self.d[L.obs_point])          # [O, 2, 7]
        f = L.obs_K0t[:, :2]
        J = dW * f[:, :, None]
        e, ok = self.reprojection()
        act = ok & self.inlier
        n = np.hypot(e[:, 0], e[:, 1])
        k = self.huber_px
        w = np.where(n <= k, 1.0, k / np.where(n > 0, n, 1.0)) * act
        rho = np.where(n <= k, 0.5 * n * n, k * n - 0.5 * k * k)
        return e, n, act, w, rho, J

    def step(self):
        L = self.L
        e, n, act, w, rho, J = self._rows()
        e = np.where(act[:, None], e, 0.0)
        J = np.where(act[:, None, None], J, 0.0)
        st = {"energy": float(np.sum(rho * act)), "sq": float(np.sum(np.where(act, n * n, 0.0))),
              "n_active": int(act.sum())}
        st["rmse"] = float(np.sqrt(st["sq"] / max(st["n_active"], 1)))
        A, B = SV.pair_maps(L, self.poses)
        Jabs = SV.absolute_jacobian(L, J.reshape(-1, 7), A, B, self.n_frames, self.d.size)
        H, g = SV.normal_equations(Jabs, np.repeat(w, 2), e.reshape(-1))
        red = SV.Reduced(H, self.n_frames, self.damping_rel, self.pinned_frame)
        dth, dd, b = red.solve(g)
        before_p, before_d = self.poses.copy(), self.d.copy()
        R, t = G.unpack(self.poses)
        dth6 = dth.reshape(-1, 6)
        Rn, tn = G.boxplus_pose(R, t, dth6[:, :3], dth6[:, 3:])
        self.poses = G.pack(Rn, tn)
        self.d = self.d + dd
        self.last = dict(S=red.S, b=b, Hdd=red.Hdd, e=e, w=w, act=act)
        st["max_disp_px"] = RS.max_centre_displacement(L, before_p, before_d, self.poses, self.d)
        self.history.append(st)
        return st

    def run(self, max_iters, conv_px):
        k = 0
        for k in range(1, max_iters + 1):
            if self.step()["max_disp_px"] < conv_px:
                break
        return k

    def remove_outliers(self, outlier_px):
        e, ok = self.reprojection()
        n = np.hypot(e[:, 0], e[:, 1])
        self.inlier &= ok & (n <= outlier_px)

    def solve(self, max_iters, conv_px=5e-3, outlier_px=None):
        """First pass, outlier removal, second pass; returns the iteration
        counts of the passes run."""
        iters = [self.run(max_iters, conv_px)]
        if outlier_px is not None:
            self.remove_outliers(outlier_px)
            iters.append(self.run(max_iters, conv_px))
        return iters
