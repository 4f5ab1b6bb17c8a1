"""Geometry parameters of the benchmark workloads, in voxel units.

Plain numbers only: both the oracle and the HIP library build their own
descriptor from these.  Frames: vial axis +z, light travelling +y, focus
plane y = 0 at the rotation axis.

Derived parameters (the paper prints the optics of its own printers, not of
these synthetic workloads):
  * thin-lens focus distance F = (field half-width) / tan(edge chief-ray
    angle), so the chief ray of the field edge meets the stated angle;
  * aperture radius A = F * tan(6.1 deg), the 12.2 deg full divergence of the
    paper's wide-aperture experiment;
  * telecentric pupil radius = sin(6.1 deg) (sine condition).
"""
import math
import numpy as np
from .pupil import pupil_concentric_jittered

HALF_DIV = math.radians(6.1)


def _thin_lens(n_pix, edge_deg):
    F = (n_pix / 2.0) / math.tan(math.radians(edge_deg))
    return F, F * math.tan(HALF_DIV)


def workload(name, pupil_seed=0):
    """Parameter dict for a named workload.  Keys mirror the descriptor:
    nx ny nz nu nv pitch_u pitch_v n_angles projector(0 telecentric,
    1 thin lens) focus pupil n_pupil pupil_xy r_outer r_inner n_air n_glass
    n_resin alpha step flags."""
    base = dict(pitch_u=1.0, pitch_v=1.0, step=0.5, flags=0, n_air=1.0,
                n_glass=1.47, n_resin=1.49, focus=0.0, pupil=0.0)
    if name == "c1":   # 64^3, telecentric, chief ray only, index-matched
        g = dict(nx=64, ny=64, nz=64, nu=64, nv=64, n_angles=90, projector=0,
                 n_pupil=1, r_outer=32.0, r_inner=32.0, alpha=0.01)
    elif name == "c2":  # 256^3, thin lens, 16 pupil samples, refracting vial
        F, A = _thin_lens(256, 10.0)
        g = dict(nx=256, ny=256, nz=256, nu=256, nv=256, n_angles=360,
                 projector=1, focus=F, pupil=A, n_pupil=16, r_outer=120.0,
                 r_inner=112.0, alpha=0.005)
    elif name == "c3":  # 256^3 telecentric index-matched, 8 pupil samples
        g = dict(nx=256, ny=256, nz=256, nu=256, nv=256, n_angles=90,
                 projector=0, pupil=math.sin(HALF_DIV), n_pupil=8,
                 r_outer=128.0, r_inner=128.0, alpha=0.01)
    elif name == "c4":  # 512^3, thin lens up to 15 deg, 8 pupil samples
        F, A = _thin_lens(512, 15.0)
        g = dict(nx=512, ny=512, nz=512, nu=512, nv=512, n_angles=360,
                 projector=1, focus=F, pupil=A, n_pupil=8, r_outer=240.0,
                 r_inner=224.0, alpha=0.005)
    elif name == "c5":  # 128^3, c2 optics scaled, 8 pupil samples
        F, A = _thin_lens(128, 10.0)
        g = dict(nx=128, ny=128, nz=128, nu=128, nv=128, n_angles=180,
                 projector=1, focus=F, pupil=A, n_pupil=8, r_outer=60.0,
                 r_inner=56.0, alpha=0.005)
    else:
        raise KeyError(name)
    out = dict(base)
    out.update(g)
    out["pupil_xy"] = pupil_concentric_jittered(out["n_pupil"], pupil_seed)
    out["angles"] = None
    return out


def scaled(params, **kw):
    """Copy of a parameter dict with fields replaced (pupil table kept
    unless given)."""
    out = dict(params)
    out.update(kw)
    if "n_pupil" in kw and "pupil_xy" not in kw:
        out["pupil_xy"] = pupil_concentric_jittered(kw["n_pupil"], 0)
    return out


WORKLOADS = ("c1", "c2", "c3", "c4", "c5")
