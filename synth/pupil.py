"""Pupil sample tables: points in the unit disk, one pattern shared by all
pixels.  The projector turns a point rho of this table into a ray direction;
that mapping belongs to the projector, not to this module.
"""
import numpy as np
from .rng import SplitMix64


def concentric_map(a, b):
    """Shirley & Chiu's concentric square-to-disk map ("A low distortion map
    between disk and square", JGT 1997), for a, b in [0, 1)."""
    sx = 2.0 * np.asarray(a, dtype=np.float64) - 1.0
    sy = 2.0 * np.asarray(b, dtype=np.float64) - 1.0
    out = np.zeros(sx.shape + (2,))
    first = np.abs(sx) > np.abs(sy)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(first, sx, sy)
        phi = np.where(first, (np.pi / 4) * (sy / sx),
                       np.pi / 2 - (np.pi / 4) * (sx / sy))
    zero = (sx == 0) & (sy == 0)
    r = np.where(zero, 0.0, r)
    phi = np.where(zero, 0.0, phi)
    out[..., 0] = r * np.cos(phi)
    out[..., 1] = r * np.sin(phi)
    return out


def _strata(n):
    nx = int(np.floor(np.sqrt(n)))
    while n % nx:
        nx -= 1
    return nx, n // nx


def pupil_concentric_jittered(n, seed):
    """`n` pupil points: a jittered nx-by-ny stratified grid on the unit
    square (16 -> 4x4, 8 -> 2x4), mapped to the disk by the concentric map.
    n == 1 gives the chief ray (the disk centre)."""
    if n == 1:
        return np.zeros((1, 2))
    nx, ny = _strata(n)
    rng = SplitMix64(seed)
    jit = rng.uniform(2 * n).reshape(n, 2)
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    a = (ii.ravel() + jit[:, 0]) / nx
    b = (jj.ravel() + jit[:, 1]) / ny
    return concentric_map(a, b)


def pupil_hex13():
    """13-point hexagonal fill of the stop: the centre, an inner ring of six
    at radius 1/2 and an outer ring of six at radius 1 rotated by 30 deg."""
    pts = [(0.0, 0.0)]
    for ring, r, off in ((1, 0.5, 0.0), (2, 1.0, np.pi / 6)):
        for k in range(6):
            a = off + k * np.pi / 3
            pts.append((r * np.cos(a), r * np.sin(a)))
    return np.array(pts)
