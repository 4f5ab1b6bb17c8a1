"""Counter-based SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).

Output i of a stream seeded with s is mix(s + (i + 1) * 0x9E3779B97F4A7C15),
with the published finaliser constants.  Vectorised over numpy uint64, whose
arithmetic wraps modulo 2**64 exactly as the definition requires.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_outputs(seed, start, count):
    """Outputs start..start+count-1 of the SplitMix64 stream for `seed`."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GOLDEN
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Sequential view of the stream: each draw advances the counter."""

    def __init__(self, seed):
        self.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        self.counter = 0

    def next_u64(self, n):
        out = splitmix64_outputs(self.seed, self.counter, n)
        self.counter += n
        return out

    def uniform(self, n=None, low=0.0, high=1.0):
        """Doubles in [low, high) from the top 53 bits of each output."""
        k = 1 if n is None else int(n)
        u = (self.next_u64(k) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        u = low + (high - low) * u
        return float(u[0]) if n is None else u

    def integer(self, low, high):
        """One integer in [low, high] (inclusive)."""
        return int(low + min(int(self.uniform() * (high - low + 1)), high - low))

    def rotation(self):
        """Uniformly random rotation matrix (Shoemake's quaternion method)."""
        u1, u2, u3 = self.uniform(3)
        a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
        q = np.array([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                      b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)])
        x, y, z, w = q
        return np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
            [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
            [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
        ])
