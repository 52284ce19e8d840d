"""Per-frame affine brightness changes of a scene's images (input generation
only): frame f is rendered with log-gain a_f and offset b_f, I'_f = e^{a_f} I_f
+ b_f, stored as float32 like every scene image."""
import numpy as np


def brighten(images, ab):
    ab = np.asarray(ab, np.float64)
    out = np.exp(ab[:, 0])[:, None, None] * np.asarray(images, np.float64) + ab[:, 1][:, None, None]
    return out.astype(np.float32)


def seeded_ab(n_frames, seed, gain=0.15, offset=0.05, pinned=0):
    """Seeded (a_f, b_f) per frame, uniform in [-gain, gain] x [-offset, offset];
    the pinned frame keeps (0, 0)."""
    rng = np.random.default_rng(seed)
    ab = np.stack([rng.uniform(-gain, gain, n_frames), rng.uniform(-offset, offset, n_frames)], 1)
    if pinned >= 0:
        ab[pinned] = 0.0
    return ab
