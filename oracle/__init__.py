"""FP64 CPU oracle of the ray-traced projector pair -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps `liboracle.so` (plain C++, FP64, std::thread)
built from `vam_oracle.cpp`; it shares no code with the HIP library.
"""
import ctypes
import math
import os

import numpy as np

from .build import LIB, build

_lib = None


class OracleGeometry(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("n_angles", ctypes.c_int32), ("projector", ctypes.c_int32),
        ("n_pupil", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("pitch_u", ctypes.c_double), ("pitch_v", ctypes.c_double),
        ("focus", ctypes.c_double), ("pupil", ctypes.c_double),
        ("r_outer", ctypes.c_double), ("r_inner", ctypes.c_double),
        ("n_air", ctypes.c_double), ("n_glass", ctypes.c_double),
        ("n_resin", ctypes.c_double), ("alpha", ctypes.c_double),
        ("step", ctypes.c_double),
        ("angles", ctypes.POINTER(ctypes.c_double)),
        ("pupil_xy", ctypes.POINTER(ctypes.c_double)),
    ]


# ray record layout (FP64), mirrors the enum in vam_oracle.cpp
R_O, R_D0, R_X1, R_D1, R_E, R_DR = 0, 3, 6, 9, 12, 15
R_T1, R_T2, R_L, R_K, R_W, R_HIT, R_COS1, R_COS2 = 18, 19, 20, 21, 22, 23, 24, 25
R_SIZE = 26

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        G = ctypes.POINTER(OracleGeometry)
        sig = {
            "oracle_record_size": (ctypes.c_int, []),
            "oracle_fresnel": (ctypes.c_double, [ctypes.c_double] * 4 + [_D, _D]),
            "oracle_refract": (ctypes.c_int, [ctypes.c_double, ctypes.c_double,
                                              _D, _D, _D, _D, _D]),
            "oracle_cylinder_roots": (ctypes.c_int, [_D, _D, ctypes.c_double, _D, _D]),
            "oracle_air_ray": (None, [G, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D]),
            "oracle_trace_ray": (None, [G, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]),
            "oracle_trace": (None, [G, _D, ctypes.c_int]),
            "oracle_forward": (None, [G, _D, ctypes.c_int, ctypes.c_int, _D, ctypes.c_int]),
            "oracle_forward_pixels": (None, [G, _D, ctypes.c_int64, _I32, _I32, _I32,
                                             _D, ctypes.c_int]),
            "oracle_adjoint": (None, [G, _D, ctypes.c_int, ctypes.c_int, _D, ctypes.c_int]),
            "oracle_count_samples": (ctypes.c_int64, [G, ctypes.c_int, ctypes.c_int,
                                                      ctypes.c_int]),
            "oracle_loss_grad": (ctypes.c_double, [G, _D, _D, ctypes.c_double,
                                                   ctypes.c_double, _D, _D, ctypes.c_int]),
            "oracle_thin_lens_magnification": (ctypes.c_double, [ctypes.c_double] * 2),
            "oracle_paraxial_etendue": (ctypes.c_double, [ctypes.c_double] * 2),
            "oracle_iris_divergence_deg": (ctypes.c_double, [ctypes.c_double] * 2),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        assert L.oracle_record_size() == R_SIZE
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(_D)


def default_threads():
    """Worker threads for the oracle: the host's cores, at most 16 (the CPU
    share of one GPU on a shared box)."""
    return max(1, min(16, os.cpu_count() or 1))


def _nt(n):
    return n if n and n > 0 else default_threads()


class Geometry:
    """Oracle geometry built from a workload parameter dict (synth.configs).
    Keeps the numpy arrays the struct points into alive."""

    def __init__(self, p):
        self.p = dict(p)
        self.pupil_xy = np.ascontiguousarray(np.asarray(p["pupil_xy"], dtype=np.float64).reshape(-1, 2))
        assert self.pupil_xy.shape[0] == p["n_pupil"]
        ang = p.get("angles")
        self.angles = None if ang is None else np.ascontiguousarray(ang, dtype=np.float64)
        s = OracleGeometry()
        for k in ("nx", "ny", "nz", "nu", "nv", "n_angles", "projector", "n_pupil", "flags"):
            setattr(s, k, int(p[k]))
        for k in ("pitch_u", "pitch_v", "focus", "pupil", "r_outer", "r_inner",
                  "n_air", "n_glass", "n_resin", "alpha", "step"):
            setattr(s, k, float(p[k]))
        s.angles = _dptr(self.angles) if self.angles is not None else _D()
        s.pupil_xy = _dptr(self.pupil_xy)
        self.s = s
        self.vol_shape = (p["nz"], p["ny"], p["nx"])
        self.n_rays = p["nu"] * p["nv"] * p["n_pupil"]

    @property
    def ref(self):
        return ctypes.byref(self.s)

    def angle(self, a):
        if self.angles is not None:
            return float(self.angles[a])
        return 2.0 * math.pi * a / self.p["n_angles"]


def trace(geom, nthreads=0):
    """All ray records, shape (nv, nu, n_pupil, R_SIZE)."""
    p = geom.p
    out = np.zeros((p["nv"], p["nu"], p["n_pupil"], R_SIZE))
    lib().oracle_trace(geom.ref, _dptr(out), _nt(nthreads))
    return out


def trace_ray(geom, u, v, j):
    out = np.zeros(R_SIZE)
    lib().oracle_trace_ray(geom.ref, u, v, j, _dptr(out))
    return out


def forward(geom, vol, a0=0, na=None, nthreads=0):
    """Projections [na, nv, nu] (FP64) of `vol` (nz, ny, nx)."""
    p = geom.p
    na = p["n_angles"] - a0 if na is None else na
    v = np.ascontiguousarray(vol, dtype=np.float64)
    assert v.shape == geom.vol_shape
    out = np.zeros((na, p["nv"], p["nu"]))
    lib().oracle_forward(geom.ref, _dptr(v), a0, na, _dptr(out), _nt(nthreads))
    return out


def forward_pixels(geom, vol, ang, vv, uu, nthreads=0):
    v = np.ascontiguousarray(vol, dtype=np.float64)
    ang = np.ascontiguousarray(ang, dtype=np.int32)
    vv = np.ascontiguousarray(vv, dtype=np.int32)
    uu = np.ascontiguousarray(uu, dtype=np.int32)
    out = np.zeros(len(ang))
    lib().oracle_forward_pixels(geom.ref, _dptr(v), len(ang),
                                ang.ctypes.data_as(_I32), vv.ctypes.data_as(_I32),
                                uu.ctypes.data_as(_I32), _dptr(out), _nt(nthreads))
    return out


def adjoint(geom, proj, a0=0, na=None, nthreads=0):
    """Dose (nz, ny, nx) deposited by projections proj [na, nv, nu]."""
    p = geom.p
    pr = np.ascontiguousarray(proj, dtype=np.float64)
    na = pr.shape[0] if na is None else na
    assert pr.shape == (na, p["nv"], p["nu"])
    out = np.zeros(geom.vol_shape)
    lib().oracle_adjoint(geom.ref, _dptr(pr), a0, na, _dptr(out), _nt(nthreads))
    return out


def count_samples(geom, a0=0, na=None, nthreads=0):
    na = geom.p["n_angles"] - a0 if na is None else na
    return int(lib().oracle_count_samples(geom.ref, a0, na, _nt(nthreads)))


def loss_grad(geom, target, proj, kappa, thr, nthreads=0):
    """(loss, dose, grad) of the dose-threshold loss."""
    p = geom.p
    t = np.ascontiguousarray(target, dtype=np.float64)
    pr = np.ascontiguousarray(proj, dtype=np.float64)
    dose = np.zeros(geom.vol_shape)
    grad = np.zeros((p["n_angles"], p["nv"], p["nu"]))
    loss = lib().oracle_loss_grad(geom.ref, _dptr(t), _dptr(pr), kappa, thr,
                                  _dptr(dose), _dptr(grad), _nt(nthreads))
    return loss, dose, grad


def fresnel(n1, n2, cos_i, cos_t):
    rs, rp = ctypes.c_double(), ctypes.c_double()
    T = lib().oracle_fresnel(n1, n2, cos_i, cos_t, ctypes.byref(rs), ctypes.byref(rp))
    return T, rs.value, rp.value


def refract(n1, n2, d, nrm):
    d = np.ascontiguousarray(d, dtype=np.float64)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    out = np.zeros(3)
    ci, ct = ctypes.c_double(), ctypes.c_double()
    rc = lib().oracle_refract(n1, n2, _dptr(d), _dptr(nrm), _dptr(out),
                              ctypes.byref(ci), ctypes.byref(ct))
    return (None if rc else out), ci.value, ct.value


def cylinder_roots(o, d, R):
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    ok = lib().oracle_cylinder_roots(_dptr(o), _dptr(d), R, ctypes.byref(lo), ctypes.byref(hi))
    return (lo.value, hi.value) if ok else None


def thin_lens_magnification(f, s_i):
    return lib().oracle_thin_lens_magnification(f, s_i)


def paraxial_etendue(pixel, full_div_deg):
    return lib().oracle_paraxial_etendue(pixel, full_div_deg)


def iris_divergence_deg(iris, f):
    return lib().oracle_iris_divergence_deg(iris, f)
