"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them compares the oracle with
itself: each checks a closed form, an exact physical invariant, a brute-force
second code path, or a number printed in the paper.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import synth
from synth.configs import scaled

HERE = os.path.dirname(os.path.abspath(__file__))


def _geom(**kw):
    p = dict(nx=16, ny=16, nz=16, nu=16, nv=16, pitch_u=1.0, pitch_v=1.0,
             n_angles=4, projector=0, focus=0.0, pupil=0.0, n_pupil=1,
             flags=0, r_outer=7.0, r_inner=7.0, n_air=1.0, n_glass=1.47,
             n_resin=1.49, alpha=0.0, step=0.5, angles=None)
    p.update(kw)
    if "pupil_xy" not in kw:
        p["pupil_xy"] = synth.pupil_concentric_jittered(p["n_pupil"], 3)
    return p


def _c2_small(n=32, n_pupil=4, **kw):
    """c2 optics scaled to an n^3 grid: thin lens with 10 deg edge chief
    ray, 12.2 deg full divergence, refracting vial."""
    F = (n / 2) / math.tan(math.radians(10))
    p = _geom(nx=n, ny=n, nz=n, nu=n, nv=n, projector=1, focus=F,
              pupil=F * math.tan(math.radians(6.1)), n_pupil=n_pupil,
              r_outer=0.47 * n, r_inner=0.44 * n, alpha=0.02, n_angles=3)
    p.update(kw)
    if "pupil_xy" not in kw:
        p["pupil_xy"] = synth.pupil_concentric_jittered(p["n_pupil"], 5)
    return p


# ------------------------------------------------------------- P14 paper --

def test_paper_printed_numbers():
    g = json.load(open(os.path.join(HERE, "golden", "paper_numbers.json")))
    tl = g["thin_lens"]
    m = oracle.thin_lens_magnification(tl["focal_length_mm"], tl["focus_distance_mm"])
    # DMD pitch x magnification = printed image pixel (4 significant figures)
    assert tl["dmd_pitch_mm"] * m == pytest.approx(tl["image_pixel_mm"], rel=5e-4)
    assert m == pytest.approx(5.0, abs=5e-3)
    # voxel = 4 image pixels in both printers
    f = g["downsample"]["factor"]
    assert f * tl["image_pixel_mm"] == pytest.approx(tl["voxel_mm"], rel=1e-12)
    tc = g["telecentric"]
    assert f * tc["dmd_pitch_mm"] * tc["magnification"] == pytest.approx(tc["voxel_mm"], rel=1e-12)
    # the printed etendue, 4 significant figures
    et = g["etendue"]
    G = oracle.paraxial_etendue(et["pixel_mm"], et["full_divergence_deg"])
    assert float("%.4g" % G) == et["etendue_sr_mm2"]
    # both (iris, divergence) pairs fit one relay focal length within the
    # printed rounding (1.9 deg: +-0.05, 12.2 deg: +-0.05)
    def f_of(iris, div):
        return 0.5 * iris / math.tan(math.radians(div / 2))
    lo = max(f_of(tc["iris_small_mm"], tc["full_divergence_small_deg"] + 0.05),
             f_of(tc["iris_large_mm"], tc["full_divergence_large_deg"] + 0.05))
    hi = min(f_of(tc["iris_small_mm"], tc["full_divergence_small_deg"] - 0.05),
             f_of(tc["iris_large_mm"], tc["full_divergence_large_deg"] - 0.05))
    assert lo < hi
    fm = 0.5 * (lo + hi)
    assert round(oracle.iris_divergence_deg(tc["iris_large_mm"], fm), 1) == tc["full_divergence_large_deg"]
    assert round(oracle.iris_divergence_deg(tc["iris_small_mm"], fm), 1) == tc["full_divergence_small_deg"]


# -------------------------------------------------------- P7 Fresnel -----

def test_fresnel_normal_incidence_brewster_symmetry():
    for n1, n2 in ((1.0, 1.47), (1.47, 1.49), (1.0, 1.49969)):
        T, rs, rp = oracle.fresnel(n1, n2, 1.0, 1.0)
        assert T == pytest.approx(1 - ((n1 - n2) / (n1 + n2)) ** 2, abs=1e-15)
    assert oracle.fresnel(1.0, 1.47, 1.0, 1.0)[0] == pytest.approx(0.963792, abs=5e-7)
    # Brewster angle: tan(theta_B) = n2 / n1 gives r_p = 0
    n1, n2 = 1.0, 1.47
    tb = math.atan(n2 / n1)
    tt = math.asin(n1 * math.sin(tb) / n2)
    _, _, rp = oracle.fresnel(n1, n2, math.cos(tb), math.cos(tt))
    assert abs(rp) < 1e-15
    # reciprocity: same T in both directions for the same angle pair
    for th in np.linspace(0.05, 1.3, 9):
        t2 = math.asin(n1 * math.sin(th) / n2)
        Ta = oracle.fresnel(n1, n2, math.cos(th), math.cos(t2))[0]
        Tb = oracle.fresnel(n2, n1, math.cos(t2), math.cos(th))[0]
        assert Ta == pytest.approx(Tb, abs=1e-15)
    # grazing incidence transmits nothing
    assert oracle.fresnel(1.0, 1.47, 0.0, math.sqrt(1 - 1 / 1.47 ** 2))[0] == pytest.approx(0.0, abs=1e-15)


# ------------------------------------------------- P5 Snell / P6 reverse --

def _c2_records(n=32, n_pupil=4):
    p = _c2_small(n, n_pupil)
    g = oracle.Geometry(p)
    return p, oracle.trace(g)


def _normal(x):
    r = math.hypot(x[0], x[1])
    return np.array([x[0] / r, x[1] / r, 0.0])


def test_snell_unit_coplanar_every_interface():
    p, R = _c2_records()
    hit = R[..., 23] == 1
    assert hit.sum() > 1000
    checked = 0
    for rec in R[hit].reshape(-1, 26):
        d0, x1, d1, e, dr = rec[3:6], rec[6:9], rec[9:12], rec[12:15], rec[15:18]
        for (dn, dt, x, n1, n2) in ((d0, d1, x1, p["n_air"], p["n_glass"]),
                                    (d1, dr, e, p["n_glass"], p["n_resin"])):
            nh = _normal(x)
            assert np.linalg.norm(dt) == pytest.approx(1.0, abs=1e-14)
            s_in = np.linalg.norm(np.cross(dn, nh))
            s_out = np.linalg.norm(np.cross(dt, nh))
            assert n1 * s_in == pytest.approx(n2 * s_out, abs=1e-14)
            assert abs(np.dot(dt, np.cross(dn, nh))) < 1e-14
            # refracted ray continues inward
            assert np.dot(dt, nh) < 0
            checked += 1
        # points lie on their cylinders
        assert math.hypot(x1[0], x1[1]) == pytest.approx(p["r_outer"], abs=1e-12)
        assert math.hypot(e[0], e[1]) == pytest.approx(p["r_inner"], abs=1e-12)
    assert checked > 2000


def test_refraction_invariants_along_path():
    """n d_z (z-translation symmetry) and n (r x d)_z (rotation symmetry
    about the vial axis) are conserved through every cylindrical wall."""
    p, R = _c2_records(48, 4)
    hit = R[..., 23] == 1
    recs = R[hit].reshape(-1, 26)
    o, d0, e, dr = recs[:, 0:3], recs[:, 3:6], recs[:, 12:15], recs[:, 15:18]
    na, nr = p["n_air"], p["n_resin"]
    np.testing.assert_allclose(na * d0[:, 2], nr * dr[:, 2], rtol=0, atol=1e-13)
    Jair = na * (o[:, 0] * d0[:, 1] - o[:, 1] * d0[:, 0])
    Jres = nr * (e[:, 0] * dr[:, 1] - e[:, 1] * dr[:, 0])
    np.testing.assert_allclose(Jair, Jres, rtol=0, atol=1e-12)


def test_reversibility():
    """The reversed resin ray, refracted back out through both walls, lands
    on the original air ray."""
    p, R = _c2_records(32, 4)
    hit = R[..., 23] == 1
    recs = R[hit].reshape(-1, 26)[::7]
    for rec in recs:
        o, d0, x1, d1, e, dr = (rec[0:3], rec[3:6], rec[6:9], rec[9:12],
                                rec[12:15], rec[15:18])
        back_g, _, _ = oracle.refract(p["n_resin"], p["n_glass"], -dr, -_normal(e))
        np.testing.assert_allclose(back_g, -d1, atol=1e-13)
        lo, hi = oracle.cylinder_roots(e, back_g, p["r_outer"])
        x1b = e + hi * back_g
        np.testing.assert_allclose(x1b, x1, atol=1e-11)
        back_a, _, _ = oracle.refract(p["n_glass"], p["n_air"], back_g, -_normal(x1b))
        np.testing.assert_allclose(back_a, -d0, atol=1e-13)
        # x1b lies on the original air line through o with direction d0
        w = x1b - o
        assert np.linalg.norm(w - np.dot(w, d0) * d0) < 1e-11


def test_central_column_closed_form():
    """Ray in the yz-plane through the axis, air tilt theta: resin
    d_z = n_air sin(theta) / n_resin, chord L = 2 R_i / sqrt(1 - d_z^2), T
    from the two incidence angles, and with V = 1 the projection is the
    attenuated geometric series of the samples."""
    s = math.sin(math.radians(5.0))
    n = 33
    p = _geom(nx=n, ny=n, nz=65, nu=n, nv=1, n_pupil=1, pupil=s,
              pupil_xy=np.array([[0.0, 1.0]]), r_outer=14.0, r_inner=12.5,
              alpha=0.03, n_angles=1, angles=np.array([0.37]))
    g = oracle.Geometry(p)
    u = (n - 1) // 2
    rec = oracle.trace_ray(g, u, 0, 0)
    th = math.asin(s)
    dz = p["n_air"] * s / p["n_resin"]
    assert rec[17] == pytest.approx(dz, abs=1e-15)
    L = 2 * p["r_inner"] / math.sqrt(1 - dz * dz)
    assert rec[20] == pytest.approx(L, abs=1e-12)
    # incidence at the outer wall: theta; in glass sin = n_air s / n_glass
    sg = p["n_air"] * s / p["n_glass"]
    T1 = oracle.fresnel(p["n_air"], p["n_glass"], math.cos(th), math.sqrt(1 - sg * sg))[0]
    sr = p["n_air"] * s / p["n_resin"]
    T2 = oracle.fresnel(p["n_glass"], p["n_resin"], math.sqrt(1 - sg * sg), math.sqrt(1 - sr * sr))[0]
    assert rec[18] == pytest.approx(T1, abs=1e-15)
    assert rec[19] == pytest.approx(T2, abs=1e-15)
    K = math.floor(L / p["step"] + 0.5)
    assert rec[21] == K
    vol = np.ones(g.vol_shape)
    P = oracle.forward(g, vol)
    a, ds = p["alpha"], p["step"]
    expect = T1 * T2 * ds * math.exp(-a * ds / 2) * (1 - math.exp(-a * K * ds)) / (1 - math.exp(-a * ds))
    assert P[0, 0, u] == pytest.approx(expect, rel=1e-13)


def test_grazing_classification():
    """A ray reaches the resin iff its impact parameter in the glass is
    below R_i (conserved angular momentum), checked away from equality."""
    n = 40
    p = _c2_small(n, 4, nu=n, pitch_u=1.5, r_outer=17.0, r_inner=15.0)
    g = oracle.Geometry(p)
    R = oracle.trace(g)
    decided = 0
    for v in range(0, p["nv"], 3):
        for u in range(p["nu"]):
            for j in range(p["n_pupil"]):
                rec = R[v, u, j]
                o, d = rec[0:3], rec[3:6]
                J = p["n_air"] * (o[0] * d[1] - o[1] * d[0])
                b_air = abs(J / p["n_air"]) / math.hypot(d[0], d[1])
                dgz = p["n_air"] * d[2] / p["n_glass"]
                b_glass = abs(J / p["n_glass"]) / math.sqrt(1 - dgz * dgz)
                crit = b_air < p["r_outer"] and b_glass < p["r_inner"]
                margin = min(abs(b_air - p["r_outer"]), abs(b_glass - p["r_inner"]))
                if margin < 1e-9:
                    continue
                assert bool(rec[23]) == crit
                decided += 1
    assert decided > 1000
    assert (R[..., 23] == 0).sum() > 100   # some rays do miss


def test_thin_lens_focus():
    p = _c2_small(24, 7)
    g = oracle.Geometry(p)
    for (u, v) in ((0, 0), (5, 17), (23, 11), (12, 12)):
        Q = np.array([(u - 11.5), 0.0, (v - 11.5)])
        for j in range(p["n_pupil"]):
            rec = oracle.trace_ray(g, u, v, j)
            o, d = rec[0:3], rec[3:6]
            w = Q - o
            assert np.linalg.norm(w - np.dot(w, d) * d) < 1e-12
            # the ray leaves its stop point on the lens plane y = -F
            t = (-p["focus"] - o[1]) / d[1]
            P = o + t * d
            rho = p["pupil_xy"][j] * p["pupil"]
            np.testing.assert_allclose([P[0], P[2]], rho, atol=1e-10)
    # chief ray (stop centre) passes through the lens centre
    pc = dict(p, n_pupil=1, pupil_xy=np.zeros((1, 2)))
    gc = oracle.Geometry(pc)
    for (u, v) in ((0, 0), (20, 3)):
        rec = oracle.trace_ray(gc, u, v, 0)
        o, d = rec[0:3], rec[3:6]
        w = np.array([0, -p["focus"], 0]) - o
        assert np.linalg.norm(w - np.dot(w, d) * d) < 1e-10


# --------------------------------------------------- P1 mass conservation --

@pytest.mark.parametrize("m", [1, 2, 4])
def test_mass_conservation_quarter_turns(m):
    """Unit pitch, chief rays only, no walls, alpha = 0, step 1/m: the
    samples of a unit tent at spacing 1/m sum to m exactly, so every voxel's
    mass is collected once per quarter-turn angle."""
    n = 20
    t, prims = synth.random_config1_target(n, 9.0, seed=m)
    p = _geom(nx=n, ny=n, nz=n, nu=n, nv=n, r_outer=9.5, r_inner=9.5,
              step=1.0 / m, n_angles=4, angles=np.array([0, 0.5, 1.0, 1.5]) * math.pi)
    rng = synth.SplitMix64(11)
    vol = t * rng.uniform(t.size).reshape(t.shape)
    # keep the support 2 voxels inside the resin
    z, y, x = np.meshgrid(*(np.arange(n) - (n - 1) / 2,) * 3, indexing="ij")
    vol[np.hypot(x, y) > 9.5 - 2] = 0
    P = oracle.forward(oracle.Geometry(p), vol)
    for a in range(4):
        assert P[a].sum() == pytest.approx(vol.sum(), rel=1e-12)


@pytest.mark.parametrize("m", [1, 2])
def test_adjoint_of_ones_is_the_angle_count(m):
    """Transpose of the pin above, voxel by voxel: with pixel centres on the
    voxel lattice and samples every 1/m along the ray, the tent weights of
    one angle's samples around any voxel add up to exactly 1 (one in each
    axis), so depositing a projection of ones gives n_angles at every voxel
    whose stencil samples all lie in the resin."""
    n = 20
    p = _geom(nx=n, ny=n, nz=n, nu=n, nv=n, r_outer=9.5, r_inner=9.5,
              step=1.0 / m, n_angles=4, angles=np.array([0, 0.5, 1.0, 1.5]) * math.pi)
    D = oracle.adjoint(oracle.Geometry(p), np.ones((4, n, n)))
    z, y, x = np.meshgrid(*(np.arange(n) - (n - 1) / 2,) * 3, indexing="ij")
    inside = np.hypot(x, y) < 9.5 - 2
    assert inside.sum() > 1000
    np.testing.assert_allclose(D[inside], 4.0, rtol=1e-12)
    # and outside the resin nothing is deposited
    assert np.all(D[np.hypot(x, y) > 9.5 + 1.5] == 0.0)


def test_mass_conservation_fails_off_lattice():
    """Control: with a step that is not 1/m, mass is not conserved to 1e-12
    (so the pin above is not vacuous)."""
    n = 20
    t, _ = synth.random_config1_target(n, 9.0, seed=1)
    p = _geom(nx=n, ny=n, nz=n, nu=n, nv=n, r_outer=9.5, r_inner=9.5,
              step=0.7, n_angles=1)
    P = oracle.forward(oracle.Geometry(p), t)
    assert abs(P[0].sum() / t.sum() - 1) > 1e-6


# ------------------------------------------------ P2 constant volume -----

@pytest.mark.parametrize("optics", ["telecentric", "thinlens"])
def test_constant_volume_geometric_series(optics):
    if optics == "telecentric":
        p = _geom(nx=32, ny=32, nz=64, nu=24, nv=12, n_pupil=5, pupil=0.1,
                  r_outer=13.0, r_inner=12.0, alpha=0.05, n_angles=2,
                  angles=np.array([0.3, 2.0]))
    else:
        p = _c2_small(32, 4, nz=64, nv=12, r_outer=13.5, r_inner=12.0,
                      alpha=0.05, n_angles=2, angles=np.array([0.1, 1.1]))
    g = oracle.Geometry(p)
    R = oracle.trace(g)
    P = oracle.forward(g, np.ones(g.vol_shape))
    a, ds = p["alpha"], p["step"]
    K = R[..., 21]
    per_ray = R[..., 22] * ds * math.exp(-a * ds / 2) * (1 - np.exp(-a * K * ds)) / (1 - math.exp(-a * ds))
    expect = per_ray.sum(axis=2)
    assert (R[..., 23] == 1).sum() > 100
    for ai in range(2):
        np.testing.assert_allclose(P[ai], expect, rtol=1e-13, atol=1e-14)


# -------------------------------------------------- P3 Radon limit -------

def _radon_setup(n, alpha_total=2.0):
    p = _geom(nx=n, ny=n, nz=n, nu=n, nv=n, r_outer=0.45 * n, r_inner=0.45 * n,
              alpha=alpha_total / n, n_angles=2, angles=np.array([0.0, 0.65]))
    return p


def _lab_ray_frame(p, theta):
    """Telecentric chief rays along +y at (x_u, z_v); entry s = 0 on the
    resin cylinder."""
    xs = (np.arange(p["nu"]) - (p["nu"] - 1) / 2) * p["pitch_u"]
    zs = (np.arange(p["nv"]) - (p["nv"] - 1) / 2) * p["pitch_v"]
    X, Z = np.meshgrid(xs, zs)            # [v, u]
    R = p["r_inner"]
    inside = np.abs(X) < R
    ey = -np.sqrt(np.maximum(R * R - X * X, 0))
    return X, Z, ey, inside


def test_radon_limit_sphere_attenuated_chords():
    errs = []
    for n in (32, 64, 128):
        p = _radon_setup(n)
        r = 0.3 * n
        c_vol = np.array([0.05, -0.08, 0.03]) * n
        vol = synth.primitive_target((n, n, n), [{"kind": "sphere", "centre": c_vol, "r": r}])
        P = oracle.forward(oracle.Geometry(p), vol)
        num = den = 0.0
        for ai, th in enumerate(p["angles"]):
            cl = np.array([math.cos(th) * c_vol[0] - math.sin(th) * c_vol[1],
                           math.sin(th) * c_vol[0] + math.cos(th) * c_vol[1], c_vol[2]])
            X, Z, ey, inside = _lab_ray_frame(p, th)
            d2 = (X - cl[0]) ** 2 + (Z - cl[2]) ** 2
            half = np.sqrt(np.maximum(r * r - d2, 0))
            s_in = (cl[1] - half) - ey
            a = p["alpha"]
            exact = np.where(d2 < r * r, np.exp(-a * s_in) * (1 - np.exp(-a * 2 * half)) / a, 0.0)
            exact = np.where(inside, exact, 0.0)
            num += np.sum((P[ai] - exact) ** 2)
            den += np.sum(exact ** 2)
        errs.append(math.sqrt(num / den))
    order = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[1] < 0.02, errs
    assert min(order) >= 0.8, (errs, order)


def test_radon_limit_gaussian_blob_second_order():
    errs = []
    for n in (32, 64, 128):
        p = _radon_setup(n)
        sig = 0.06 * n
        c_vol = np.array([0.02, -0.03, 0.01]) * n
        vol = synth.gaussian_blob_volume((n, n, n), c_vol, sig)
        P = oracle.forward(oracle.Geometry(p), vol)
        num = den = 0.0
        a = p["alpha"]
        for ai, th in enumerate(p["angles"]):
            cl = np.array([math.cos(th) * c_vol[0] - math.sin(th) * c_vol[1],
                           math.sin(th) * c_vol[0] + math.cos(th) * c_vol[1], c_vol[2]])
            X, Z, ey, inside = _lab_ray_frame(p, th)
            d2 = (X - cl[0]) ** 2 + (Z - cl[2]) ** 2
            s_c = cl[1] - ey
            exact = (np.exp(-d2 / (2 * sig * sig)) * sig * math.sqrt(2 * math.pi)
                     * math.exp(a * a * sig * sig / 2) * np.exp(-a * s_c))
            exact = np.where(inside, exact, 0.0)
            num += np.sum((P[ai] - exact) ** 2)
            den += np.sum(exact ** 2)
        errs.append(math.sqrt(num / den))
    order = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[2] < 2e-3, errs
    assert min(order) >= 1.8, (errs, order)


# ----------------------------------------------- P11 adjoint identity ----

@pytest.mark.parametrize("kind", ["c1", "optics"])
def test_adjoint_identity(kind):
    if kind == "c1":
        p = scaled(synth.workload("c1"), n_angles=12)
    else:
        p = _c2_small(24, 3, n_angles=5)
    g = oracle.Geometry(p)
    rng = synth.SplitMix64(99)
    x = rng.uniform(int(np.prod(g.vol_shape))).reshape(g.vol_shape)
    y = rng.uniform(p["n_angles"] * p["nv"] * p["nu"]).reshape(p["n_angles"], p["nv"], p["nu"])
    Ax = oracle.forward(g, x)
    Aty = oracle.adjoint(g, y)
    lhs, rhs = np.sum(Ax * y), np.sum(x * Aty)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)


# ------------------------------------------------------ P12 symmetries ---

def test_quarter_turn_symmetry():
    n = 24
    p = _c2_small(n, 3, angles=np.array([0.4, 0.4 + math.pi / 2]), n_angles=2)
    g = oracle.Geometry(p)
    rng = synth.SplitMix64(5)
    V = rng.uniform(n ** 3).reshape(n, n, n)
    P = oracle.forward(g, V)
    # V'(p) = V(Rz(-90deg) p) = V(y, -x): V'[z, j, i] = V[z, n-1-i, j]
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")   # [j, i]
    Vr = V[:, n - 1 - I, J]
    P2 = oracle.forward(g, Vr)
    np.testing.assert_allclose(P[1], P2[0], rtol=1e-12, atol=1e-12 * np.abs(P).max())


def test_mirror_symmetry():
    n = 24
    p = _c2_small(n, 3, angles=np.array([0.7]), n_angles=1)
    pm = dict(p)
    pm["pupil_xy"] = p["pupil_xy"] * np.array([-1.0, 1.0])
    pm["angles"] = np.array([-0.7])
    rng = synth.SplitMix64(6)
    V = rng.uniform(n ** 3).reshape(n, n, n)
    P = oracle.forward(oracle.Geometry(p), V)
    Pm = oracle.forward(oracle.Geometry(pm), V[:, :, ::-1])
    np.testing.assert_allclose(P[0], Pm[0][:, ::-1], rtol=1e-12, atol=1e-12 * np.abs(P).max())


# ------------------------------------------------- P13 brute force 8^3 ---

def test_brute_force_dense_matrix_straight_rays():
    p = _geom(nx=8, ny=8, nz=8, nu=8, nv=6, n_pupil=3, pupil=0.15,
              r_outer=4.2, r_inner=4.2, alpha=0.07, step=0.5, n_angles=3,
              pitch_u=0.9, pitch_v=1.1, angles=np.array([0.0, 0.9, 2.5]))
    g = oracle.Geometry(p)
    A = brute.dense_matrix(p, brute.straight_rays(p), p["angles"])
    rng = synth.SplitMix64(8)
    V = rng.uniform(512).reshape(8, 8, 8)
    Y = rng.uniform(3 * 6 * 8).reshape(3, 6, 8)
    np.testing.assert_allclose(oracle.forward(g, V).ravel(), A @ V.ravel(), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(oracle.adjoint(g, Y).ravel(), A.T @ Y.ravel(), rtol=1e-13, atol=1e-14)


def test_brute_force_dense_matrix_refracting_thin_lens():
    p = _c2_small(8, 3, nu=8, nv=8, r_outer=4.3, r_inner=3.8, alpha=0.06,
                  n_angles=2, angles=np.array([0.2, 4.0]))
    g = oracle.Geometry(p)
    rays = brute.rays_from_records(p, oracle.trace(g))
    assert len(rays) > 50
    A = brute.dense_matrix(p, rays, p["angles"])
    rng = synth.SplitMix64(9)
    V = rng.uniform(512).reshape(8, 8, 8)
    Y = rng.uniform(2 * 64).reshape(2, 8, 8)
    np.testing.assert_allclose(oracle.forward(g, V).ravel(), A @ V.ravel(), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(oracle.adjoint(g, Y).ravel(), A.T @ Y.ravel(), rtol=1e-13, atol=1e-14)


def test_brute_force_continuum_integral_second_order():
    """The sampled ray sums converge to the continuous integral of the
    interpolated volume at second order in the step.  The interpolant has
    kinks at cell faces, whose midpoint-rule errors fluctuate in sign from
    step to step, so the order is the least-squares slope of the RMS error
    over many rays and five steps."""
    n = 8
    angs = np.array([0.3, 1.4, 2.9])
    base = _geom(nx=n, ny=n, nz=n, nu=n, nv=n, r_outer=4.5, r_inner=4.5,
                 alpha=0.1, n_angles=3, angles=angs)
    V = synth.gaussian_blob_volume((n, n, n), (0.3, -0.2, 0.1), 1.2)
    z, y, x = np.meshgrid(*(np.arange(n) - (n - 1) / 2,) * 3, indexing="ij")
    V[np.hypot(x, y) > 2.3] = 0.0     # zero near the wall: no end effects
    R = oracle.trace(oracle.Geometry(base))
    exact = np.zeros((3, 6, 6))
    for a in range(3):
        for v in range(1, 7):
            for u in range(1, 7):
                rec = R[v, u, 0]
                exact[a, v - 1, u - 1] = brute.continuum_ray_integral(
                    base, V, rec[12:15], rec[15:18], rec[20], rec[22], angs[a], sub=96)
    hs = [0.5, 0.25, 0.125, 0.0625, 0.03125]
    errs = []
    for ds in hs:
        P = oracle.forward(oracle.Geometry(dict(base, step=ds)), V)
        errs.append(np.sqrt(np.mean((P[:, 1:7, 1:7] - exact) ** 2)))
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert slope > 1.6, (errs, slope)
    assert errs[-1] < errs[0] / 50, errs


# -------------------------------------------- pixel subset = full result --

def test_forward_pixels_match_full_rows():
    p = _c2_small(16, 3)
    g = oracle.Geometry(p)
    rng = synth.SplitMix64(12)
    V = rng.uniform(16 ** 3).reshape(16, 16, 16)
    P = oracle.forward(g, V)
    a = np.array([0, 1, 2, 2]); v = np.array([3, 8, 15, 0]); u = np.array([1, 9, 4, 15])
    np.testing.assert_array_equal(oracle.forward_pixels(g, V, a, v, u), P[a, v, u])


def test_count_samples_matches_trace():
    p = scaled(synth.workload("c1"), n_angles=3)
    g = oracle.Geometry(p)
    R = oracle.trace(g)
    # every c1 sample lies inside the grid's stencil range, so the count is
    # sum of K over rays times the angles
    assert oracle.count_samples(g) == 3 * int(R[..., 21].sum())


@pytest.mark.parametrize("kind", ["straight", "refracting"])
def test_count_samples_brute_force_rays_leaving_the_grid(kind):
    """The sample count (the throughput metric's denominator) where rays
    leave the grid: the resin is wider than the grid in x and y, and tilted
    rays leave through the top and bottom, so some samples have no voxel
    in reach and others reach it with only part of their stencil.  Counted
    by brute force against every voxel centre."""
    if kind == "straight":
        p = _geom(nx=9, ny=8, nz=7, nu=14, nv=10, n_pupil=3, pupil=0.35,
                  r_outer=6.5, r_inner=6.5, step=0.5, n_angles=3,
                  pitch_u=0.95, pitch_v=1.05, angles=np.array([0.0, 0.61, 2.2]))
        rays = brute.straight_rays(p)
    else:
        p = _c2_small(10, 3, nu=16, nv=14, nz=8, r_outer=7.4, r_inner=6.9, step=0.45,
                      n_angles=3, angles=np.array([0.3, 1.9, 4.4]))
        rays = brute.rays_from_records(p, oracle.trace(oracle.Geometry(p)))
    g = oracle.Geometry(p)
    n_all = sum(int(math.floor(r[4] / p["step"] + 0.5)) for r in rays) * len(p["angles"])
    want = brute.count_samples(p, rays, p["angles"])
    got = oracle.count_samples(g)
    # the case is one that exercises the rule: many samples fall outside
    assert 0 < want < 0.8 * n_all, (want, n_all)
    assert got == want
    # and per angle
    for a in range(len(p["angles"])):
        assert oracle.count_samples(g, a, 1) == brute.count_samples(p, rays, p["angles"][a:a + 1])
