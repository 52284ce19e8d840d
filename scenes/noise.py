"""Seeded 3-D value noise used to texture the synthetic scenes.

Lattice values are uniform in [0, 1) and looked up through a seeded
permutation hash; they are blended with the quintic fade curve
6t^5 - 15t^4 + 10t^3 (C2-continuous, so rendered images have smooth
gradients). Octaves double the frequency and halve the amplitude; the sum is
divided by the total amplitude so the texture stays in [0, 1].
"""
import numpy as np


class ValueNoise3:
    def __init__(self, seed, table=256):
        rng = np.random.default_rng(seed)
        self.mask = table - 1
        self.perm = rng.permutation(table).astype(np.int64)
        self.vals = rng.random(table)
        # lattice value reached through the last hash step, and int32 copies
        # (exact integer arithmetic: the same values as _lattice, fewer gathers)
        self._p32 = self.perm.astype(np.int32)
        self._vp = self.vals[self.perm]

    def _lattice(self, i, j, k):
        p, m = self.perm, self.mask
        h = p[(p[(p[i & m] + j) & m] + k) & m]
        return self.vals[h]

    @staticmethod
    def _fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def single(self, x, y, z):
        xi, yi, zi = np.floor(x), np.floor(y), np.floor(z)
        fx, fy, fz = self._fade(x - xi), self._fade(y - yi), self._fade(z - zi)
        m, p = self.mask, self._p32
        # the table size is a power of two, so masking the low bits of the int32
        # lattice indices gives the same hash as masking int64 ones
        i, j, k = xi.astype(np.int32), yi.astype(np.int32), zi.astype(np.int32)
        out = 0.0
        for di in (0, 1):
            wx = fx if di else 1.0 - fx
            hi = p[(i + di) & m]
            for dj in (0, 1):
                wy = fy if dj else 1.0 - fy
                hij = p[(hi + j + dj) & m]
                for dk in (0, 1):
                    wz = fz if dk else 1.0 - fz
                    out = out + wx * wy * wz * self._vp[(hij + k + dk) & m]
        return out

    def fractal(self, pts, base_freq=4.0, octaves=3):
        """pts: [..., 3] world points -> texture in [0, 1]."""
        x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
        total, amp, freq, norm = 0.0, 1.0, base_freq, 0.0
        for o in range(octaves):
            # a per-octave offset decorrelates the lattices of successive octaves
            off = 17.31 * (o + 1)
            total = total + amp * self.single(x * freq + off, y * freq + 2 * off, z * freq + 3 * off)
            norm += amp
            amp *= 0.5
            freq *= 2.0
        return total / norm
