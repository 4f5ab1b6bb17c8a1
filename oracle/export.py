"""8-bit projection export (FP64, numpy) -- TEST INFRASTRUCTURE.

Sec. 2.7: projection values more than three standard deviations above the
mean (over all pixels of all angles) are clipped, and the range is rescaled
to the 8-bit grey levels sent to the projector.  Reading: population
standard deviation, clip = mean + 3 std, negatives to 0, level =
round-half-even(255 x / clip) with the product in FP64.
"""
import numpy as np


def export_stats(proj):
    x = np.asarray(proj, dtype=np.float64).ravel()
    mean = x.mean()
    sd = x.std()
    return mean, sd, mean + 3.0 * sd


def equalize_u8(proj, stats=None):
    x = np.asarray(proj, dtype=np.float64)
    mean, sd, clip = export_stats(x) if stats is None else stats
    if clip <= 0:
        return np.zeros(x.shape, dtype=np.uint8), (mean, sd, clip)
    v = np.rint(np.minimum(np.maximum(x, 0.0), clip) * (255.0 / clip))
    return np.clip(v, 0, 255).astype(np.uint8), (mean, sd, clip)
