"""Exact planar test problem (input generation only).

A fronto-parallel plane Z = Z0 in front of host frame 0 carries an intensity
that is affine in the host's pixel coordinates. Every other frame is the host
translated (no rotation). For this geometry the target images are also affine
in their own pixels, so bilinear interpolation and central differences are
exact at every pyramid level (the 2x2 box average of an affine image is the
same affine function at the coarse pixel centre). Brightness constancy then
holds exactly at the true parameters.
"""
import numpy as np

from .configs import PATTERN8, Scene


def planar(seed=0, width=96, height=64, n_frames=3, n_points=40, z0=2.0, n_levels=1, f=90.0,
           translations=None, coef=(0.45, 2.0e-3, 1.3e-3)):
    rng = np.random.default_rng(seed)
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    K = np.array([f, f, cx, cy])
    a, b, c = coef
    if translations is None:
        translations = [np.zeros(3)] + [np.array([0.08 * k, -0.03 * k, 0.05 * k]) for k in range(1, n_frames)]
    vv, uu = np.mgrid[0:height, 0:width].astype(np.float64)
    imgs = []
    for t in translations:
        # host pixel u that lands on target pixel u': u - c = ((u' - c)(Z0 + tz) - f tx) / Z0
        uh = ((uu - cx) * (z0 + t[2]) - f * t[0]) / z0 + cx
        vh = ((vv - cy) * (z0 + t[2]) - f * t[1]) / z0 + cy
        imgs.append(a + b * uh + c * vh)
    images = np.stack(imgs)
    poses = np.zeros((n_frames, 12))
    for k, t in enumerate(translations):
        poses[k, :9] = np.eye(3).reshape(-1)
        poses[k, 9:] = t
    margin = 5 * 2 ** (n_levels - 1) + 2
    us = rng.integers(margin, width - margin, size=n_points)
    vs = rng.integers(margin, height - margin, size=n_points)
    obs_ptr = np.arange(n_points + 1, dtype=np.int32) * (n_frames - 1)
    obs_frame = np.tile(np.arange(1, n_frames, dtype=np.int32), n_points)
    d = np.full(n_points, 1.0 / z0)
    return Scene(
        name="planar", images=images, intrinsics=np.tile(K, (n_frames, 1)), poses_gt=poses,
        poses_init=poses.copy(), host_frame=np.zeros(n_points, np.int32),
        host_uv=np.stack([us, vs], 1).astype(np.float32), inv_depth_gt=d, inv_depth_init=d.copy(),
        obs_ptr=obs_ptr, obs_frame=obs_frame, n_levels=n_levels, pattern=PATTERN8.copy(),
        meta={"seed": seed},
    )
