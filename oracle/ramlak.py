"""Ram-Lak filtering of projection rows (FP64, numpy) -- TEST INFRASTRUCTURE.

The discrete band-limited ramp filter for sample spacing tau (Ramachandran &
Lakshminarayanan 1971; Kak & Slaney, "Principles of Computerized
Tomographic Imaging", ch. 3): h(0) = 1/(4 tau^2), h(n tau) = 0 for even
n != 0, h(n tau) = -1/(n^2 pi^2 tau^2) for odd n; the filtered projection is
Q(n tau) = tau sum_k h(k tau) P((n - k) tau), taken over the row (zero
outside), then clipped at zero for the plain initialisation of Sec. 2.3.
"""
import numpy as np


def ramlak_kernel(half_width, tau=1.0):
    """h(n tau) for n = -half_width .. half_width."""
    n = np.arange(-half_width, half_width + 1)
    h = np.zeros(n.shape, dtype=np.float64)
    h[n == 0] = 1.0 / (4.0 * tau * tau)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (n[odd].astype(np.float64) ** 2 * np.pi ** 2 * tau * tau)
    return n, h


def ramlak_filter(rows, tau=1.0, clip_negative=True):
    """Filter every row (last axis) of `rows`; plain direct convolution."""
    rows = np.asarray(rows, dtype=np.float64)
    nu = rows.shape[-1]
    flat = rows.reshape(-1, nu)
    n, h = ramlak_kernel(nu - 1, tau)
    out = np.zeros_like(flat)
    for i in range(flat.shape[0]):
        # full convolution, then the nu outputs aligned with the input
        full = np.convolve(flat[i], h)
        out[i] = tau * full[nu - 1: 2 * nu - 1]
    if clip_negative:
        out = np.maximum(out, 0.0)
    return out.reshape(rows.shape)
