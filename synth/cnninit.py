"""Seeded initial parameters of the learned-initialiser network.

He-normal weights (Gaussian, std sqrt(2 / fan_in), fan_in = 9 c_in) for all
but the last convolution, whose weights and bias start at zero so that the
untrained network returns its residual input unchanged.  Normals come from
SplitMix64 uniforms by the Box-Muller transform.  Layout per layer:
W[c_out][3][3][c_in], then b[c_out].
"""
import numpy as np

from .rng import SplitMix64


def layer_shapes(layers, channels):
    """(c_in, c_out) of each convolution: 2 inputs, 1 output."""
    return [(2 if l == 0 else channels, 1 if l == layers - 1 else channels) for l in range(layers)]


def param_count(layers, channels):
    return sum(co * 9 * ci + co for ci, co in layer_shapes(layers, channels))


def normals(rng, n):
    u1 = rng.uniform(n)
    u2 = rng.uniform(n)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


def he_init(layers, channels, seed, zero_last=True):
    rng = SplitMix64(seed)
    out = []
    shapes = layer_shapes(layers, channels)
    for l, (ci, co) in enumerate(shapes):
        nw = co * 9 * ci
        if zero_last and l == len(shapes) - 1:
            out.append(np.zeros(nw + co))
        else:
            out.append(normals(rng, nw) * np.sqrt(2.0 / (9 * ci)))
            out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)
