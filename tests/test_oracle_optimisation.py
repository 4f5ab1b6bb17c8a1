"""Pins of the oracle's optimisation pieces: the dose-threshold gradient
(central finite differences on a 16^3 crop) and the Ram-Lak filter (its
frequency response and filtered back-projection of a smooth blob)."""
import math

import numpy as np
import pytest

import oracle
from oracle import ramlak
import synth


def _geom16(**kw):
    n = 16
    F = (n / 2) / math.tan(math.radians(10))
    p = dict(nx=n, ny=n, nz=n, nu=n, nv=n, pitch_u=1.0, pitch_v=1.0, n_angles=6,
             projector=1, focus=F, pupil=F * math.tan(math.radians(6.1)), n_pupil=3,
             flags=0, r_outer=7.5, r_inner=7.0, n_air=1.0, n_glass=1.47, n_resin=1.49,
             alpha=0.02, step=0.5, angles=None)
    p.update(kw)
    p["pupil_xy"] = synth.pupil_concentric_jittered(p["n_pupil"], 2)
    return p


def test_loss_gradient_central_differences_16cube():
    p = _geom16()
    g = oracle.Geometry(p)
    t, _ = synth.random_config1_target(16, 6.0, seed=3)
    P = oracle.forward(g, t)
    D = oracle.adjoint(g, P)
    g0 = P / np.percentile(D[t > 0], 50)
    kappa, thr = 20.0, 0.8
    loss, _, grad = oracle.loss_grad(g, t, g0, kappa, thr)
    rng = synth.SplitMix64(4)
    idx = np.flatnonzero(np.abs(grad) > 1e-3 * np.abs(grad).max())
    pick = idx[(rng.uniform(12) * len(idx)).astype(int)]
    h = 1e-4 * float(np.abs(g0).max())
    for i in pick:
        gp = g0.copy().ravel(); gp[i] += h
        gm = g0.copy().ravel(); gm[i] -= h
        lp = oracle.loss_grad(g, t, gp.reshape(g0.shape), kappa, thr)[0]
        lm = oracle.loss_grad(g, t, gm.reshape(g0.shape), kappa, thr)[0]
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(grad.ravel()[i], rel=1e-5, abs=1e-9 * np.abs(grad).max())


def test_ramlak_frequency_response_is_the_ramp():
    n, h = ramlak.ramlak_kernel(4096, 1.0)
    for f in (0.05, 0.13, 0.25, 0.37, 0.45):
        H = np.sum(h * np.cos(2 * np.pi * f * n))
        assert H == pytest.approx(f, abs=2e-4)


def test_filtered_back_projection_recovers_a_blob():
    """Parallel rays, no attenuation or walls: the oracle's forward is the
    Radon transform and its adjoint the back-projection, so Ram-Lak filtering
    between them (without clipping) reconstructs a smooth volume."""
    n = 32
    na = 120
    p = dict(nx=n, ny=n, nz=4, nu=n, nv=4, pitch_u=1.0, pitch_v=1.0, n_angles=na, projector=0,
             focus=0.0, pupil=0.0, n_pupil=1, flags=0, r_outer=15.5, r_inner=15.5, n_air=1.0,
             n_glass=1.0, n_resin=1.0, alpha=0.0, step=0.25, angles=None,
             pupil_xy=np.zeros((1, 2)))
    g = oracle.Geometry(p)
    vol = synth.gaussian_blob_volume((4, n, n), (1.5, -2.0, 0.0), 3.0)
    vol = np.repeat(vol[1:2], 4, axis=0)     # z-invariant slab
    sino = oracle.forward(g, vol)
    q = ramlak.ramlak_filter(sino, 1.0, clip_negative=False)
    rec = oracle.adjoint(g, q) * (np.pi / na)
    mid = slice(1, 3)
    err = np.linalg.norm(rec[mid] - vol[mid]) / np.linalg.norm(vol[mid])
    assert err < 0.05, err
