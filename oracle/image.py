"""Image functions (oracle, FP64, test infrastructure).

The paper treats every image function I(.) as the bilinear interpolation of
its pixel grid (Notation). Conventions used throughout (the paper gives none):
  * pixel centres sit at integer coordinates; u is the column, v the row;
  * level l+1 of the pyramid is the 2x2 box average of level l, size
    floor(W/2) x floor(H/2); its intrinsics are f/2 and (c + 0.5)/2 - 0.5,
    which keeps a level-(l+1) pixel centre on the centre of its 2x2 block;
  * the image gradient is the central difference on the grid, bilinearly
    interpolated between pixel centres (the paper's grad I0 of a bilinear
    image is undefined at pixel centres);
  * a sample position is usable when u in [1, W-3] and v in [1, H-3], which
    keeps the bilinear 2x2 footprint and its central-difference neighbours
    inside the image.
"""
import numpy as np


def pyramid(images, n_levels):
    """images [F][H][W] -> list of FP64 stacks, level 0 first."""
    lv = [np.asarray(images, np.float64)]
    for _ in range(1, n_levels):
        a = lv[-1]
        h, w = a.shape[1] // 2, a.shape[2] // 2
        a = a[:, : 2 * h, : 2 * w]
        lv.append(0.25 * (a[:, 0::2, 0::2] + a[:, 0::2, 1::2] + a[:, 1::2, 0::2] + a[:, 1::2, 1::2]))
    return lv


def level_intrinsics(K, level):
    """K [..., 4] = (fx, fy, cx, cy) at level 0 -> the same at `level`."""
    K = np.asarray(K, float)
    s = 2.0 ** level
    return np.stack([K[..., 0] / s, K[..., 1] / s, (K[..., 2] + 0.5) / s - 0.5, (K[..., 3] + 0.5) / s - 0.5], -1)


def level_pixel(uv, level):
    """A level-0 pixel position expressed in level-`level` pixels."""
    return (np.asarray(uv, float) + 0.5) / 2.0 ** level - 0.5


def central_gradients(stack):
    """Central differences (I[i, j+1] - I[i, j-1]) / 2 and (I[i+1, j] - I[i-1, j]) / 2;
    zero on the one-pixel border (never sampled: see `in_bounds`)."""
    gu = np.zeros_like(stack)
    gv = np.zeros_like(stack)
    gu[:, :, 1:-1] = 0.5 * (stack[:, :, 2:] - stack[:, :, :-2])
    gv[:, 1:-1, :] = 0.5 * (stack[:, 2:, :] - stack[:, :-2, :])
    return gu, gv


def in_bounds(u, v, width, height):
    return (u >= 1.0) & (u <= width - 3.0) & (v >= 1.0) & (v <= height - 3.0)


def bilinear(stack, frame, u, v):
    """Bilinear interpolation of stack[frame] at (u, v); callers guarantee in-bounds
    positions (out-of-bounds entries are clamped and must be masked by the caller)."""
    H, W = stack.shape[1], stack.shape[2]
    u = np.clip(u, 0.0, W - 2.0)
    v = np.clip(v, 0.0, H - 2.0)
    j0 = np.floor(u).astype(np.int64)
    i0 = np.floor(v).astype(np.int64)
    j0 = np.minimum(j0, W - 2)
    i0 = np.minimum(i0, H - 2)
    a = u - j0
    b = v - i0
    f = np.asarray(frame, np.int64)
    return ((1 - a) * (1 - b) * stack[f, i0, j0] + a * (1 - b) * stack[f, i0, j0 + 1]
            + (1 - a) * b * stack[f, i0 + 1, j0] + a * b * stack[f, i0 + 1, j0 + 1])
