"""Parity of the HIP projector pair with the FP64 oracle, through the C ABI.

Tolerances.  FP32 results: relative L2 error <= 1e-5 against the FP64 oracle
on the same seeded inputs.  Reduced-precision storage: one rounding of the
stored volume and one of the stored projection, so rel-L2 <= 2 u with
u = 2^-8 (BF16) or 2^-11 (FP16); binary targets are exact in both.
Ray-table fields are FP64 on both sides and must agree to 1e-12.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth.configs import scaled

torch = pytest.importorskip("torch")
import paper_2211_03516_amd as vam

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relL2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


def maxrel(x, ref):
    """Largest element-wise deviation, relative to the largest |ref|."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def check(x, ref, tol=1e-5, what=""):
    """rel-L2 <= tol and every element within tol of the largest |ref|."""
    e2, em = relL2(x, ref), maxrel(x, ref)
    say("%s rel-L2 %.3e, max element error %.3e of max |ref|" % (what, e2, em))
    assert np.isfinite(np.asarray(x, dtype=np.float64)).all()
    assert e2 <= tol and em <= tol, (what, e2, em)
    return e2


def c2_small(n=64, n_pupil=16, n_angles=24, **kw):
    """c2 optics scaled to n^3: thin lens, 10 deg edge chief ray, 12.2 deg
    divergence, refracting vial."""
    F = (n / 2) / math.tan(math.radians(10))
    p = scaled(synth.workload("c2"), nx=n, ny=n, nz=n, nu=n, nv=n, focus=F,
               pupil=F * math.tan(math.radians(6.1)), n_pupil=n_pupil,
               r_outer=0.47 * n, r_inner=0.44 * n, alpha=0.02, n_angles=n_angles)
    p.update(kw)
    return p


def gpu_geom(p):
    say("setup geometry", {k: p[k] for k in ("nx", "ny", "nz", "nu", "nv", "n_pupil", "n_angles", "projector")})
    g = vam.Geometry(p)
    torch.cuda.synchronize()
    return g


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


# ------------------------------------------------------------- ray table --

@pytest.mark.parametrize("name", ["c1", "c2small", "c2"])
def test_ray_table_matches_oracle_trace(name):
    p = synth.workload("c1") if name == "c1" else (c2_small() if name == "c2small" else synth.workload("c2"))
    g = gpu_geom(p)
    R = g.export_rays()                        # (np, nv, nu, 12)
    O = oracle.trace(oracle.Geometry(p))       # (nv, nu, np, 26)
    O = np.transpose(O, (2, 0, 1, 3))
    hit = O[..., oracle.R_HIT] == 1
    np.testing.assert_array_equal(R[..., 11] == 1, hit)
    say(name, "rays hit", int(hit.sum()), "of", hit.size)
    np.testing.assert_allclose(R[hit][:, 0:3], O[hit][:, oracle.R_E:oracle.R_E + 3], rtol=0, atol=1e-12)
    np.testing.assert_allclose(R[hit][:, 3:6], O[hit][:, oracle.R_DR:oracle.R_DR + 3], rtol=0, atol=1e-13)
    np.testing.assert_allclose(R[hit][:, 6], O[hit][:, oracle.R_L], rtol=1e-12, atol=1e-11)
    np.testing.assert_array_equal(R[hit][:, 7], O[hit][:, oracle.R_K])
    np.testing.assert_allclose(R[hit][:, 8], O[hit][:, oracle.R_W], rtol=1e-13, atol=0)
    rays_hit, samples = g.stats()
    assert rays_hit == int(hit.sum())
    if name != "c2":
        assert samples == oracle.count_samples(oracle.Geometry(p))
    g.close()


# ----------------------------------------------------------- small parity --

def _parity_case(p, vol, proj_in, tol=1e-5):
    og = oracle.Geometry(p)
    g = gpu_geom(p)
    say("forward parity", p["nx"], p["n_angles"])
    Pg = g.forward(to_dev(vol)).cpu().numpy()
    Po = oracle.forward(og, vol)
    e_f = relL2(Pg, Po)
    say("adjoint parity", p["nx"], p["n_angles"])
    Dg = g.back(to_dev(proj_in)).cpu().numpy()
    Do = oracle.adjoint(og, proj_in)
    e_a = relL2(Dg, Do)
    say("rel-L2 forward %.3e adjoint %.3e; max element error forward %.3e adjoint %.3e"
        % (e_f, e_a, maxrel(Pg, Po), maxrel(Dg, Do)))
    assert np.isfinite(Pg).all() and np.isfinite(Dg).all()
    assert e_f <= tol and e_a <= tol
    assert maxrel(Pg, Po) <= tol and maxrel(Dg, Do) <= tol
    return g, og, Pg, Po


@pytest.mark.parametrize("m", [1, 2])
def test_mass_conservation_and_adjoint_of_ones(m):
    # closed forms, no oracle: telecentric chief rays on the voxel lattice,
    # no walls, alpha = 0, step 1/m, quarter turns.  The samples of a unit
    # tent at spacing 1/m sum to m, so each angle's projection sums to the
    # volume's sum, and the deposit of a projection of ones is the number of
    # angles at every voxel 2 voxels inside the resin (zero outside it);
    # 40^3 spans several lab boxes.
    n, R = 40, 19.5
    p = dict(nx=n, ny=n, nz=n, nu=n, nv=n, pitch_u=1.0, pitch_v=1.0, n_angles=4,
             angles=np.array([0.0, 0.5, 1.0, 1.5]) * math.pi, projector=0, focus=0.0, pupil=0.0,
             n_pupil=1, pupil_xy=None, flags=0, r_outer=R, r_inner=R, n_air=1.0, n_glass=1.47,
             n_resin=1.49, alpha=0.0, step=1.0 / m)
    g = gpu_geom(p)
    z, y, x = np.meshgrid(*(np.arange(n) - (n - 1) / 2,) * 3, indexing="ij")
    rho = np.hypot(x, y)
    rng = synth.SplitMix64(21 + m)
    vol = rng.uniform(n ** 3).reshape(n, n, n)
    vol[rho > R - 2] = 0.0
    P = g.forward(to_dev(vol)).double().cpu().numpy()
    sums = P.reshape(4, -1).sum(axis=1) / vol.sum()
    D = g.back(to_dev(np.ones((4, n, n)))).double().cpu().numpy()
    inside = rho < R - 2
    say("m %d: projection sums / volume sum %s; deposit of ones inside: %.7f .. %.7f"
        % (m, np.array2string(sums, precision=8), D[inside].min(), D[inside].max()))
    assert np.all(np.abs(sums - 1.0) <= 1e-6)
    np.testing.assert_allclose(D[inside], 4.0, rtol=1e-6)
    assert np.all(D[rho > R + 1.5] == 0.0)
    g.close()


def test_constant_volume_geometric_series():
    # closed form, no oracle: V = 1 everywhere, telecentric chief rays, no
    # walls, alpha > 0.  Every sample's trilinear value is 1, so a pixel at
    # lateral offset x collects the geometric series
    #   step e^{-alpha step/2} (1 - e^{-alpha K step}) / (1 - e^{-alpha step})
    # with K = floor(2 sqrt(R^2 - x^2) / step + 1/2), the same at any angle.
    n, R, alpha, step = 48, 20.0, 0.05, 0.5
    angles = np.array([0.0, 0.3, 1.1, 2.0, 3.7, 5.5])
    p = dict(nx=n, ny=n, nz=n, nu=n, nv=n, pitch_u=1.0, pitch_v=1.0, n_angles=len(angles), angles=angles,
             projector=0, focus=0.0, pupil=0.0, n_pupil=1, pupil_xy=np.zeros((1, 2)), flags=0, r_outer=R,
             r_inner=R, n_air=1.0, n_glass=1.47, n_resin=1.49, alpha=alpha, step=step)
    g = gpu_geom(p)
    P = g.forward(to_dev(np.ones((n, n, n)))).double().cpu().numpy()
    xu = np.arange(n) - (n - 1) / 2
    L = 2.0 * np.sqrt(np.maximum(R * R - xu * xu, 0.0))
    K = np.floor(L / step + 0.5)
    q = math.exp(-alpha * step)
    want = step * math.exp(-alpha * step / 2) * (1.0 - q ** K) / (1.0 - q)
    rows = slice(1, n - 1)   # rows whose stencil stays inside the grid in z
    err = np.abs(P[:, rows, :] - want[None, None, :]).max() / want.max()
    say("geometric series: max error %.2e of the largest pixel (%.4f)" % (err, want.max()))
    assert err <= 2e-6
    g.close()


def _fresnel_unpolarised(n1, n2, cos_i):
    """Transmittance (mean of s and p) and cos of the refracted angle."""
    cos_t = math.sqrt(1.0 - (n1 / n2) ** 2 * (1.0 - cos_i * cos_i))
    rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t)
    rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t)
    return 1.0 - 0.5 * (rs * rs + rp * rp), cos_t


def test_central_column_closed_form():
    # closed form, no oracle: thin lens, refracting vial, chief rays, V = 1.
    # The chief ray of the centre column (odd grid) lies in the plane through
    # the vial axis, so it stays there through both walls; its incidence
    # angles are its tilt and the refracted tilt, and its resin chord is
    # 2 R_i / cos(tilt in the resin).  The pixel collects T1 T2 times the
    # attenuated geometric series of that chord, at every angle.
    n = 49
    F = (n / 2) / math.tan(math.radians(10))
    p = dict(nx=n, ny=n, nz=n, nu=n, nv=n, pitch_u=1.0, pitch_v=1.0, n_angles=3,
             angles=np.array([0.0, 2.3, 4.0]), projector=1, focus=F, pupil=F * math.tan(math.radians(6.1)),
             n_pupil=1, pupil_xy=np.zeros((1, 2)), flags=0, r_outer=0.47 * n, r_inner=0.44 * n, n_air=1.0,
             n_glass=1.47, n_resin=1.49, alpha=0.02, step=0.5)
    want = []
    for v in range(n):
        z = v - (n - 1) / 2
        T1, c1 = _fresnel_unpolarised(p["n_air"], p["n_glass"], F / math.hypot(F, z))
        T2, c2 = _fresnel_unpolarised(p["n_glass"], p["n_resin"], c1)
        K = math.floor(2.0 * p["r_inner"] / c2 / p["step"] + 0.5)
        q = math.exp(-p["alpha"] * p["step"])
        want.append(T1 * T2 * p["step"] * math.exp(-p["alpha"] * p["step"] / 2) * (1.0 - q ** K) / (1.0 - q))
    want = np.array(want)
    g = gpu_geom(p)
    P = g.forward(to_dev(np.ones((n, n, n)))).double().cpu().numpy()
    rows = slice(5, n - 5)   # the ray's z drift keeps its stencil inside the grid
    err = np.abs(P[:, rows, n // 2] - want[None, rows]).max() / want.max()
    say("central column: max error %.2e of the largest pixel (%.4f)" % (err, want.max()))
    assert err <= 2e-6
    g.close()


def test_c1_full_forward_and_adjoint():
    p = synth.workload("c1")
    t, _ = synth.random_config1_target(64, 32.0, seed=0)
    Po = oracle.forward(oracle.Geometry(p), t)
    g, og, Pg, _ = _parity_case(p, t, Po)
    # seeded U[0,1) inputs too
    rng = synth.SplitMix64(1)
    x = rng.uniform(64 ** 3).reshape(64, 64, 64)
    y = rng.uniform(90 * 64 * 64).reshape(90, 64, 64)
    check(g.forward(to_dev(x)).cpu().numpy(), oracle.forward(og, x), what="c1 U[0,1) forward")
    check(g.back(to_dev(y)).cpu().numpy(), oracle.adjoint(og, y), what="c1 U[0,1) deposit")
    g.close()


def test_vial_wider_than_the_grid():
    # the resin (R_i 28) is wider than the 48^3 grid (half-width 24) and the
    # thin-lens rays tilt out through the top and bottom, so samples leave
    # the grid sideways at angle-dependent places: parity of both operators
    # and the exact sample count (samples whose stencil touches the grid)
    p = c2_small(48, n_pupil=4, n_angles=9, r_outer=31.0, r_inner=28.0)
    rng = synth.SplitMix64(41)
    x = rng.uniform(48 ** 3).reshape(48, 48, 48)
    y = rng.uniform(9 * 48 * 48).reshape(9, 48, 48)
    g, og, *_ = _parity_case(p, x, y)
    _, samples = g.stats()
    want = oracle.count_samples(og)
    say("samples per pass: library %d, oracle %d" % (samples, want))
    assert samples == want
    g.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_c2_optics_64(seed):
    p = c2_small()
    t, _ = synth.random_config2_target(64, p["r_inner"], seed=seed)
    rng = synth.SplitMix64(100 + seed)
    y = rng.uniform(p["n_angles"] * 64 * 64).reshape(p["n_angles"], 64, 64)
    g, *_ = _parity_case(p, t, y)
    g.close()


def test_ragged_sizes_and_telecentric_pupil():
    # sizes that are not multiples of the 64 x 4 lane tile, odd everything
    p = scaled(synth.workload("c3"), nx=37, ny=41, nz=29, nu=70, nv=5, n_angles=7,
               r_outer=18.0, r_inner=16.5, n_pupil=3, pitch_u=0.6, pitch_v=1.3)
    rng = synth.SplitMix64(7)
    x = rng.uniform(29 * 41 * 37).reshape(29, 41, 37)
    y = rng.uniform(7 * 5 * 70).reshape(7, 5, 70)
    g, *_ = _parity_case(p, x, y)
    g.close()


def test_chief_ray_only_null_pupil_and_no_fresnel():
    p = c2_small(32, n_pupil=1, n_angles=5, flags=vam.VAM_NO_FRESNEL)
    p["pupil_xy"] = None
    po = dict(p, pupil_xy=np.zeros((1, 2)))
    rng = synth.SplitMix64(8)
    x = rng.uniform(32 ** 3).reshape(32, 32, 32)
    g = gpu_geom(p)
    Pg = g.forward(to_dev(x)).cpu().numpy()
    check(Pg, oracle.forward(oracle.Geometry(po), x))
    g.close()


def test_rays_missing_the_vial():
    # most pixel columns lie beside a thin vial: those rays carry nothing
    p = scaled(synth.workload("c1"), nx=16, ny=16, nz=16, nu=16, nv=4,
               r_outer=3.0, r_inner=3.0, n_angles=3)
    g = gpu_geom(p)
    hits, samples = g.stats()
    assert 0 < hits < 16 * 4
    x = torch.ones((16, 16, 16), device=DEV)
    P = g.forward(x).cpu().numpy()
    Po = oracle.forward(oracle.Geometry(p), np.ones((16, 16, 16)))
    assert np.isfinite(P).all()
    check(P, Po)
    assert (P[:, :, :5] == 0).all() and (P[:, :, -5:] == 0).all()
    g.close()
    # a vial narrower than half a pixel: every ray misses
    p2 = dict(p, r_outer=0.2, r_inner=0.2, nu=2, nv=2)
    g2 = gpu_geom(p2)
    assert g2.stats() == (0, 0)
    assert np.abs(g2.forward(x).cpu().numpy()).max() == 0
    d = g2.back(torch.ones((3, 2, 2), device=DEV)).cpu().numpy()
    assert np.abs(d).max() == 0
    g2.close()


def test_zero_inputs_and_single_pixel_dmd():
    # all-zero volume / projections give exact zeros on every default path;
    # a 1 x 1 DMD with one angle still matches the oracle
    p = c2_small(24, n_pupil=4, n_angles=3)
    g = gpu_geom(p)
    assert float(g.forward(torch.zeros((24, 24, 24), device=DEV)).abs().max()) == 0.0
    assert float(g.back(torch.zeros((3, 24, 24), device=DEV)).abs().max()) == 0.0
    g.close()
    p1 = dict(c2_small(16, n_pupil=4, n_angles=1), nu=1, nv=1)
    g1 = gpu_geom(p1)
    rng = synth.SplitMix64(17)
    x = rng.uniform(16 ** 3).reshape(16, 16, 16)
    og = oracle.Geometry(p1)
    check(g1.forward(to_dev(x)).cpu().numpy(), oracle.forward(og, x))
    y = np.array([[[0.7]]])
    check(g1.back(to_dev(y)).cpu().numpy(), oracle.adjoint(og, y))
    g1.close()


# ---------------------------------------------------- API behaviour -------

def test_angle_ranges_determinism_accumulate():
    p = c2_small(32, n_pupil=4, n_angles=10)
    g = gpu_geom(p)
    rng = synth.SplitMix64(9)
    x = to_dev(rng.uniform(32 ** 3).reshape(32, 32, 32))
    full = g.forward(x)
    part = g.forward(x, angle_begin=3, angle_count=5)
    assert torch.equal(full[3:8], part)
    again = g.forward(x)
    assert torch.equal(full, again)            # deterministic forward
    y = to_dev(rng.uniform(10 * 32 * 32).reshape(10, 32, 32))
    d_all = g.back(y).double()
    d_a = g.back(y[:4], angle_begin=0)
    g.back(y[4:], out=d_a, accumulate=True, angle_begin=4)
    assert relL2(d_a.double().cpu().numpy(), d_all.cpu().numpy()) <= 1e-6
    # out-of-range and empty angle windows are rejected
    with pytest.raises(vam.VamError):
        g.forward(x, angle_begin=8, angle_count=5)
    with pytest.raises(vam.VamError):
        g.forward(x, angle_begin=2, angle_count=0)
    with pytest.raises(vam.VamError):
        g.back(y[:0], angle_begin=2)
    with pytest.raises(vam.VamError):
        g.back(y[:3], angle_begin=9)
    g.close()


def test_forward_variants_agree():
    p = c2_small(48, n_pupil=4, n_angles=12)
    g = gpu_geom(p)
    rng = synth.SplitMix64(11)
    x = rng.uniform(48 ** 3).reshape(48, 48, 48)
    ref = oracle.forward(oracle.Geometry(p), x)
    for variant in (vam.FWD_RAY, vam.FWD_PARTIALS, vam.FWD_DEFAULT):
        g.set_forward_variant(variant)
        P1 = g.forward(to_dev(x))
        P2 = g.forward(to_dev(x))
        assert torch.equal(P1, P2)              # every variant is deterministic
        check(P1.cpu().numpy(), ref, what="forward variant %d" % variant)
    with pytest.raises(vam.VamError):
        g.set_forward_variant(3)
    g.close()


def test_fixed_point_forward():
    """The default forward adds each segment's partial to its pixel as a 64-bit
    integer: a signed volume at every box edge and in BF16 / FP16, a zero
    volume, an exact power-of-two rescaling (the scale is a power of two, so
    the integers do not change), and a NaN (every value NaN)."""
    n = 44
    p = c2_small(n, n_pupil=4, n_angles=7)
    g = gpu_geom(p)
    og = oracle.Geometry(p)
    rng = synth.SplitMix64(23)
    x = rng.uniform(n ** 3).reshape(n, n, n) - 0.4
    ref = oracle.forward(og, x)
    for edge in (8, 16, 12):
        g.set_box_edge(edge)
        check(g.forward(to_dev(x)).cpu().numpy(), ref, what="fixed-point forward, edge %d, signed" % edge)
    P = g.forward(to_dev(x))
    P_big = g.forward(to_dev(x) * 2.0 ** 40)
    P_small = g.forward(to_dev(x) * 2.0 ** -40)
    assert torch.equal(P_big, P * 2.0 ** 40) and torch.equal(P_small, P * 2.0 ** -40)
    for dt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        xs = torch.from_numpy(x).to(tdt)
        check(g.forward(xs.to(DEV)).cpu().numpy(), oracle.forward(og, xs.double().numpy()),
              what="fixed-point forward, %s pairs" % dt)
    assert torch.count_nonzero(g.forward(torch.zeros(n, n, n, device=DEV))) == 0
    # high dynamic range: a block of 1e8 in a U(0, 1) volume.  The integer
    # sums against the FP32 partial sums of the same samples (variant 2):
    # every pixel above 1e-9 of the largest, those whose rays miss the block
    # included, agrees to FP32 level (an add's rounding is at most 2^-61 of
    # a bound set by the largest value); against the oracle the usual
    # element-wise bound (pixels that graze the block's faces carry the
    # samples' FP32 position rounding times the 1e8 step)
    hdr = rng.uniform(n ** 3).reshape(n, n, n)
    hdr[20:24, 18:22, 21:25] = 1e8
    Ph = g.forward(to_dev(hdr)).cpu().numpy().astype(np.float64)
    g.set_forward_lanes(1)  # the same per-segment sums as variant 2
    Ph1 = g.forward(to_dev(hdr)).cpu().numpy().astype(np.float64)
    g.set_forward_lanes(2)
    Ph2 = g.forward(to_dev(hdr)).cpu().numpy().astype(np.float64)
    g.set_forward_lanes(0)
    g.set_forward_variant(vam.FWD_PARTIALS)
    Pp = g.forward(to_dev(hdr)).cpu().numpy().astype(np.float64)
    g.set_forward_variant(vam.FWD_DEFAULT)
    sel = np.abs(Pp) >= 1e-9 * np.abs(Pp).max()
    for what, Px in (("one lane", Ph1), ("two lanes", Ph2), ("default", Ph)):
        rel = np.abs(Px - Pp)[sel] / np.abs(Pp)[sel]
        say("fixed-point forward (%s), 1e8 block in U(0, 1): %d of %d pixels, max relative difference to "
            "FP32 partial sums %.2e" % (what, sel.sum(), sel.size, rel.max()))
        assert rel.max() <= 1e-5
    check(Ph, oracle.forward(og, hdr), what="fixed-point forward, 1e8 block in U(0, 1)")
    bad = to_dev(x)
    bad[20, 3, 7] = float("nan")
    assert torch.isnan(g.forward(bad)).all()
    # the fixed-point sums are not affected by the previous call's NaN
    check(g.forward(to_dev(x)).cpu().numpy(), ref, what="fixed-point forward after a NaN")
    g.close()


def test_forward_lanes_per_segment():
    """The fixed-point forward's march modes against the oracle: two lanes
    per segment (alternate samples, each lane's Horner sum over r^2, combined
    as S_even + r S_odd), one lane, and one lane keeping its cell's LDS words
    (the same bits as one lane); signed FP32, BF16 and FP16 volumes, every
    box edge, and a strongly absorbing resin (r far from 1), where a wrong
    power of r on any part would show."""
    n = 40
    for alpha in (0.02, 0.6):
        p = c2_small(n, n_pupil=4, n_angles=5, alpha=alpha)
        g = gpu_geom(p)
        og = oracle.Geometry(p)
        rng = synth.SplitMix64(29)
        x = rng.uniform(n ** 3).reshape(n, n, n) - 0.3
        ref = oracle.forward(og, x)
        one = {}
        for lanes in (1, 2, 3):
            g.set_forward_lanes(lanes)
            for edge in (8, 16, 12):
                g.set_box_edge(edge)
                check(g.forward(to_dev(x)).cpu().numpy(), ref,
                      what="%d lanes, alpha %g, edge %d" % (lanes, alpha, edge))
            P1 = g.forward(to_dev(x))
            assert torch.equal(P1, g.forward(to_dev(x)))
            outs = {"f32": P1}
            for dt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
                xs = torch.from_numpy(x).to(tdt)
                outs[dt] = g.forward(xs.to(DEV))
                check(outs[dt].cpu().numpy(), oracle.forward(og, xs.double().numpy()),
                      what="%d lanes, alpha %g, %s pairs" % (lanes, alpha, dt))
            if lanes == 1:
                one = outs
            elif lanes == 3:
                # the cached cell words change where the values are read
                # from, not the arithmetic
                for dt in outs:
                    assert torch.equal(outs[dt], one[dt]), dt
        with pytest.raises(vam.VamError):
            g.set_forward_lanes(4)
        # the default picks by format (cached cell words for FP32 and BF16,
        # one lane for FP16): the same bits as one lane
        g.set_forward_lanes(0)
        assert torch.equal(g.forward(to_dev(x)), one["f32"])
        for dt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
            xs = torch.from_numpy(x).to(tdt).to(DEV)
            assert torch.equal(g.forward(xs), one[dt]), dt
        g.close()


def test_box_edges_agree():
    p = c2_small(48, n_pupil=4, n_angles=6)
    g = gpu_geom(p)
    rng = synth.SplitMix64(12)
    x = to_dev(rng.uniform(48 ** 3).reshape(48, 48, 48))
    y = to_dev(rng.uniform(6 * 48 * 48).reshape(6, 48, 48))
    og = oracle.Geometry(p)
    Pref = oracle.forward(og, x.double().cpu().numpy())
    Dref = oracle.adjoint(og, y.double().cpu().numpy())
    for edge in (8, 16, 12):
        g.set_box_edge(edge)
        check(g.forward(x).cpu().numpy(), Pref, what="box edge %d forward" % edge)
        check(g.back(y).cpu().numpy(), Dref, what="box edge %d deposit" % edge)
    # edges without a compiled footprint are rejected on the host
    for edge in (4, 7, 20):
        with pytest.raises(vam.VamError):
            g.set_box_edge(edge)
    check(g.forward(x).cpu().numpy(), Pref, what="after the rejected edges")
    g.close()


def test_adjoint_variants_agree():
    p = c2_small(48, n_pupil=4, n_angles=12)
    g = gpu_geom(p)
    rng = synth.SplitMix64(10)
    y = to_dev(rng.uniform(12 * 48 * 48).reshape(12, 48, 48))
    ref = oracle.adjoint(oracle.Geometry(p), y.cpu().numpy().astype(np.float64))
    for variant in (vam.ADJ_RAY, vam.ADJ_GATHER, vam.ADJ_DEFAULT):
        g.set_adjoint_variant(variant)
        check(g.back(y).cpu().numpy(), ref, what="deposit variant %d" % variant)
    with pytest.raises(vam.VamError):
        g.set_adjoint_variant(3)
    g.close()


@pytest.mark.parametrize("step", [0.3, 1.3, 2.2])
def test_box_kernels_any_step(step):
    # steps of more than one cell per sample, and many samples per cell
    p = c2_small(40, n_pupil=4, n_angles=8, step=step)
    g = gpu_geom(p)
    rng = synth.SplitMix64(14)
    x = rng.uniform(40 ** 3).reshape(40, 40, 40)
    y = rng.uniform(8 * 40 * 40).reshape(8, 40, 40)
    og = oracle.Geometry(p)
    check(g.forward(to_dev(x)).cpu().numpy(), oracle.forward(og, x), what="step %.1f forward" % step)
    check(g.back(to_dev(y)).cpu().numpy(), oracle.adjoint(og, y), what="step %.1f deposit" % step)
    g.close()


def _n_supp(p):
    """Most samples of all rays in any 4 x 4 x 3 block of lab-frame unit
    cells (x, y from -(R_i + 1), z from the padded grid's origin): the count
    the fixed-point deposit's scale is built on, from the oracle's rays."""
    R = oracle.trace(oracle.Geometry(p))
    hit = R[..., oracle.R_HIT] == 1
    e, d = R[hit][:, oracle.R_E:oracle.R_E + 3], R[hit][:, oracle.R_DR:oracle.R_DR + 3]
    K = R[hit][:, oracle.R_K].astype(np.int64)
    ray = np.repeat(np.arange(len(K)), K)
    k = np.arange(K.sum()) - np.repeat(np.cumsum(K) - K, K)
    q = e[ray] + ((k + 0.5) * p["step"])[:, None] * d[ray]
    x0, z0 = -(p["r_inner"] + 1.0), -(0.5 * (p["nz"] - 1) + 2)
    ncx, ncz = int(math.ceil(2 * (p["r_inner"] + 1.0))), p["nz"] + 4
    gz = q[:, 2] - z0
    keep = (gz >= 0.5) & (gz <= p["nz"] + 2.5)      # the samples the kernels march
    i = np.clip(np.floor(q[keep] - np.array([x0, x0, z0])).astype(np.int64), 0,
                np.array([ncx - 1, ncx - 1, ncz - 1]))
    c = np.zeros((ncz, ncx, ncx), dtype=np.int64)
    np.add.at(c, (i[:, 2], i[:, 1], i[:, 0]), 1)
    w = np.zeros_like(c)
    for dz in range(3):
        for dy in range(4):
            for dx in range(4):
                w[:ncz - dz, :ncx - dy, :ncx - dx] += c[dz:, dy:, dx:]
    return int(w.max())


def test_integer_deposit_dynamic_range_and_nonfinite():
    # fixed-point LDS sums: the scale follows each (box, angle)'s largest
    # value, so projections spanning 12 orders of magnitude across angles
    # and pixels keep FP32-level accuracy; a NaN makes the whole dose NaN
    # (the voxels' 64-bit integers cannot hold it)
    p = c2_small(40, n_pupil=4, n_angles=6)
    g = gpu_geom(p)
    rng = synth.SplitMix64(16)
    y = rng.uniform(6 * 40 * 40).reshape(6, 40, 40)
    y *= 10.0 ** (-12 * rng.uniform(6 * 40 * 40).reshape(6, 40, 40) ** 4)
    y[2] *= 1e6
    y[4, ::2] *= -1.0
    ref = oracle.adjoint(oracle.Geometry(p), y)
    D = g.back(to_dev(y)).cpu().numpy()
    check(D, ref, what="dynamic range")
    # the angles without the 1e6 factor, on their own
    y_small = y.copy()
    y_small[2] = 0.0
    check(g.back(to_dev(y_small)).cpu().numpy(), oracle.adjoint(oracle.Geometry(p), y_small),
          what="dynamic range without the large angle")
    bad = y.copy()
    bad[3, 20, 20] = float("nan")
    Db = g.back(to_dev(bad)).cpu().numpy()
    assert np.isnan(Db).all()
    # and the next call is not affected
    check(g.back(to_dev(y)).cpu().numpy(), ref, what="dynamic range after a NaN")
    g.close()


def test_fixed_point_deposit_per_voxel_bound():
    # A few bright pixels over a dim floor: a dim voxel in a box that a
    # bright ray crosses is summed at the bright ray's scale.  Per voxel the
    # fixed-point rounding is bounded by
    #   sum over angles of n_supp^2 (step / n_pupil) max_a|P| / 2^30
    # (at most n adds per angle and box, each within 1/(2S) with
    # S >= 2^30 / (n (step / n_pupil) max|P|), n <= n_supp, the largest
    # window count of all samples), plus the FP32 rounding of the sample
    # weights; every voxel is held to that bound.
    p = c2_small(40, n_pupil=4, n_angles=6)
    g = gpu_geom(p)
    rng = synth.SplitMix64(18)
    y = 1e-4 * rng.uniform(6 * 40 * 40).reshape(6, 40, 40)
    spots = (rng.uniform(36) * 40).astype(int).reshape(6, 3, 2)
    for a in range(6):
        for v, u in spots[a]:
            y[a, v, u] = 1e4
    og = oracle.Geometry(p)
    ref = oracle.adjoint(og, y)
    D = g.back(to_dev(y)).cpu().numpy().astype(np.float64)
    ns = _n_supp(p)
    quant = sum(ns * ns * (p["step"] / p["n_pupil"]) * np.abs(y[a]).max() / 2.0 ** 30 for a in range(6))
    bound = quant + 1e-6 * np.abs(ref) + 1e-7 * np.abs(ref).max()
    err = np.abs(D - ref)
    dim = (ref > 0) & (ref < 1e-3 * ref.max())
    say("n_supp %d; per-voxel bound from rounding %.3e; worst error / bound %.3e; worst relative error of "
        "dim voxels %.3e" % (ns, quant, float((err / bound).max()), float((err[dim] / ref[dim]).max())))
    assert np.all(err <= bound)
    g.close()


def test_work_orders_agree():
    # every (box, angle) item is processed exactly once in each work order
    p = c2_small(40, n_pupil=4, n_angles=10)
    g = gpu_geom(p)
    rng = synth.SplitMix64(15)
    x = rng.uniform(40 ** 3).reshape(40, 40, 40)
    y = rng.uniform(10 * 40 * 40).reshape(10, 40, 40)
    og = oracle.Geometry(p)
    Pref, Dref = oracle.forward(og, x), oracle.adjoint(og, y)
    first = None
    for blk in (0, 1, 3, 8, 64):
        g.set_angle_blocks(deposit=blk, forward=blk)
        P, D = g.forward(to_dev(x)), g.back(to_dev(y))
        ef = relL2(P.cpu().numpy(), Pref)
        ea = relL2(D.cpu().numpy(), Dref)
        say("angle block %d: forward %.3e deposit %.3e" % (blk, ef, ea))
        assert ef <= 1e-5 and ea <= 1e-5
        # integer sums per pixel and per voxel: the same bits in every order
        if first is None:
            first = (P, D)
        assert torch.equal(P, first[0]) and torch.equal(D, first[1])
    g.close()


def test_segment_orders_agree():
    # the order of the segments inside a box only decides which lanes march
    # which segment: the forward adds each segment's sum to its pixel as an
    # integer, and the deposit adds each segment's runs exactly inside a
    # workgroup and each workgroup's cells to the voxels as integers: the
    # same bits for every order
    p = c2_small(40, n_pupil=4, n_angles=10)
    g = gpu_geom(p)
    rng = synth.SplitMix64(16)
    x = to_dev(rng.uniform(40 ** 3).reshape(40, 40, 40))
    y = to_dev(rng.uniform(10 * 40 * 40).reshape(10, 40, 40))
    P0, D0 = g.forward(x), g.back(y)
    for order in range(17):
        g.set_segment_order(order)
        g.set_segment_order(order, forward=True)
        P1, D1 = g.forward(x), g.back(y)
        say("segment order %d: forward equal %s, deposit equal %s" % (order, torch.equal(P0, P1), torch.equal(D0, D1)))
        assert torch.equal(P0, P1) and torch.equal(D0, D1)
    with pytest.raises(vam.VamError):
        g.set_segment_order(17)
    g.close()


def test_gather_deposit_angles_accumulate_and_order():
    # the voxel-driven gather against the oracle on an angle sub-range, with
    # accumulation into an existing dose, and bitwise repeatable
    p = c2_small(40, n_pupil=6, n_angles=10)
    g = gpu_geom(p)
    g.set_adjoint_variant(vam.ADJ_GATHER)
    rng = synth.SplitMix64(13)
    y = rng.uniform(10 * 40 * 40).reshape(10, 40, 40)
    og = oracle.Geometry(p)
    ref = oracle.adjoint(og, y[3:8], a0=3, na=5)
    D1 = g.back(to_dev(y[3:8]), angle_begin=3)
    D2 = g.back(to_dev(y[3:8]), angle_begin=3)
    assert torch.equal(D1, D2)
    say("gather sub-range rel-L2 %.3e" % relL2(D1.cpu().numpy(), ref))
    check(D1.cpu().numpy(), ref)
    base = to_dev(rng.uniform(40 ** 3).reshape(40, 40, 40))
    acc = base.clone()
    g.back(to_dev(y[3:8]), angle_begin=3, out=acc, accumulate=True)
    check((acc - base).cpu().numpy(), ref)
    # telecentric, index-matched rays (c1 optics)
    p1 = scaled(synth.workload("c1"), n_angles=20)
    g1 = gpu_geom(p1)
    g1.set_adjoint_variant(vam.ADJ_GATHER)
    y1 = rng.uniform(20 * 64 * 64).reshape(20, 64, 64)
    e1 = relL2(g1.back(to_dev(y1)).cpu().numpy(), oracle.adjoint(oracle.Geometry(p1), y1))
    say("gather c1 rel-L2 %.3e" % e1)
    assert e1 <= 1e-5
    g1.close()
    g.close()


@pytest.mark.parametrize("dt,bound", [("bf16", 2 * 2.0 ** -8), ("f16", 2 * 2.0 ** -11)])
def test_reduced_precision_storage(dt, bound):
    tdt = torch.bfloat16 if dt == "bf16" else torch.float16
    p = c2_small(64, n_pupil=8, n_angles=16)
    t, _ = synth.random_config2_target(64, p["r_inner"], seed=3)
    og = oracle.Geometry(p)
    g = gpu_geom(p)
    P = g.forward(to_dev(t, tdt), out_dtype=tdt)
    Po = oracle.forward(og, t)
    e_f = relL2(P.float().cpu().numpy(), Po)
    # adjoint of stored reduced-precision projections (input rounding only)
    y = Po / Po.max()
    D = g.back(to_dev(y, tdt)).cpu().numpy()
    e_a = relL2(D, oracle.adjoint(og, y))
    say(dt, "rel-L2 forward %.3e adjoint %.3e bound %.3e" % (e_f, e_a, bound))
    assert e_f <= bound and e_a <= bound
    g.close()


def test_forward_dtypes_in_turn_on_one_handle():
    # the box forward stages BF16 / FP16 volumes as 16-bit pairs and FP32
    # volumes as values in the same working buffer: every call must replace
    # all of it, padding included, whatever the previous call's format
    p = c2_small(40, n_pupil=4, n_angles=6)
    g = gpu_geom(p)
    og = oracle.Geometry(p)
    rng = synth.SplitMix64(19)
    x = rng.uniform(40 ** 3).reshape(40, 40, 40)
    ref = oracle.forward(og, x)
    for dt in ("bf16", "f32", "f16", "f32", "f16", "bf16"):
        tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dt]
        xs = torch.from_numpy(x).to(tdt)
        P = g.forward(xs.to(DEV)).cpu().numpy()
        if dt == "f32":
            check(P, ref, what="fp32 after a 16-bit call")
        else:
            # against the oracle of the volume as stored: only FP32 sums
            check(P, oracle.forward(og, xs.double().numpy()), what="%s pairs" % dt)
    g.close()


# ------------------------------------------- full c2 size, sampled outputs --

@pytest.fixture(scope="module")
def c2_full():
    p = synth.workload("c2")
    t, _ = synth.random_config2_target(256, p["r_inner"], seed=0)
    g = gpu_geom(p)
    yield p, t, g
    g.close()


@pytest.mark.parametrize("variant", ["default", "ray", "partials"])
def test_c2_full_forward_sampled(c2_full, variant):
    p, t, g = c2_full
    g.set_forward_variant({"ray": vam.FWD_RAY, "partials": vam.FWD_PARTIALS}.get(variant, vam.FWD_DEFAULT))
    say("c2 full forward, 360 angles, variant", variant)
    P = g.forward(to_dev(t)).cpu().numpy()
    g.set_forward_variant(vam.FWD_DEFAULT)
    assert np.isfinite(P).all()
    rng = synth.SplitMix64(21)
    ang = np.repeat([0, 45, 137, 359], 96)
    vv = (rng.uniform(len(ang)) * 256).astype(np.int32)
    uu = (rng.uniform(len(ang)) * 256).astype(np.int32)
    ref = oracle.forward_pixels(oracle.Geometry(p), t, ang, vv, uu)
    got = P[ang, vv, uu]
    check(got, ref, what="c2 sampled forward (%d pixels)" % len(ang))


def test_c2_full_forward_full_projections(c2_full):
    # four full 256^2 projections of the benchmark's forward (all 360 angles
    # computed in one call), angles spread over the turn, pixel by pixel
    p, t, g = c2_full
    say("c2 full forward, full projections")
    P = g.forward(to_dev(t)).cpu().numpy()
    og = oracle.Geometry(p)
    for a in (0, 97, 199, 301):
        check(P[a], oracle.forward(og, t, a0=a, na=1)[0], what="c2 forward angle %d" % a)


def test_c2_full_samples_per_pass_8_angles():
    # the throughput metric's denominator at the benchmark's optics, on 8
    # angles spread over the full turn: exact integer agreement
    p = dict(synth.workload("c2"))
    p["angles"] = np.array([0, 41, 97, 150, 199, 251, 302, 353]) * (2 * math.pi / 360)
    p["n_angles"] = 8
    g = gpu_geom(p)
    _, samples = g.stats()
    g.close()
    want = oracle.count_samples(oracle.Geometry(p))
    say("c2 samples over 8 angles: library %d, oracle %d" % (samples, want))
    assert samples == want


@pytest.mark.parametrize("a", [0, 61, 137, 199, 263, 331])
def test_c2_full_adjoint_angles(c2_full, a):
    # the default deposit of one full 256^2 projection at angles spread over
    # the turn, against the oracle voxel by voxel
    p, t, g = c2_full
    rng = synth.SplitMix64(220 + a)
    y = rng.uniform(256 * 256).reshape(1, 256, 256)
    say("c2 full deposit, angle", a)
    D = g.back(to_dev(y), angle_begin=a).cpu().numpy()
    check(D, oracle.adjoint(oracle.Geometry(p), y, a0=a, na=1), what="c2 deposit angle %d" % a)


def test_c2_full_adjoint_variants_one_angle(c2_full):
    p, t, g = c2_full
    rng = synth.SplitMix64(22)
    y = rng.uniform(256 * 256).reshape(1, 256, 256)
    ref = oracle.adjoint(oracle.Geometry(p), y, a0=37, na=1)
    for variant in (vam.ADJ_RAY, vam.ADJ_GATHER):
        g.set_adjoint_variant(variant)
        say("c2 full adjoint, angle 37, variant", variant)
        D = g.back(to_dev(y), angle_begin=37).cpu().numpy()
        check(D, ref, what="c2 deposit angle 37 variant %d" % variant)
    g.set_adjoint_variant(vam.ADJ_DEFAULT)


def test_c2_full_quarter_turn_symmetry(c2_full):
    # a property that holds at any size, here the benchmark's full workload:
    # the vial turns about z, so turning the volume by 90 degrees is the same
    # as projecting 90 angles (90 degrees) later, and the deposit of angles
    # [90, 180) turned back equals the deposit of the same projections at
    # angles [0, 90)
    p, t, g = c2_full
    n = p["nx"]
    rng = synth.SplitMix64(29)
    V = to_dev(rng.uniform(n ** 3).reshape(n, n, n))
    rot = lambda a: a.transpose(1, 2).flip(2).contiguous()   # V'[z, j, i] = V[z, n-1-i, j]
    say("c2 full quarter-turn symmetry")
    P = g.forward(V)
    Pr = g.forward(rot(V))
    ef = float((P[90:].double() - Pr[:270].double()).norm() / P[90:].double().norm())
    y = torch.from_numpy(rng.uniform(90 * 256 * 256).reshape(90, 256, 256).astype(np.float32)).to(DEV)
    D90 = g.back(y, angle_begin=90).double()
    D0 = g.back(y, angle_begin=0).double()
    ed = float((rot(D90) - D0).norm() / D0.norm())
    say("forward: P[a + 90](V) vs P[a](rot V) rel-L2 %.3e; deposit: rot(D[90, 180)) vs D[0, 90) rel-L2 %.3e"
        % (ef, ed))
    assert ef <= 1e-6 and ed <= 1e-6


def test_c2_full_mirror_symmetry(c2_full):
    # a property that holds at any size: mirroring the optics in x (pupil
    # points x -> -x) and the volume in x is the same as flipping every
    # projection in u with the angles reversed (theta -> -theta); the
    # deposit follows as the transpose
    p, t, g = c2_full
    na = p["n_angles"]
    pm = dict(p)
    pm["pupil_xy"] = np.asarray(p["pupil_xy"]) * np.array([-1.0, 1.0])
    gm = gpu_geom(pm)
    perm = torch.tensor([(na - a) % na for a in range(na)], device=DEV)
    rng = synth.SplitMix64(31)
    V = to_dev(t * rng.uniform(t.size).reshape(t.shape))
    P = g.forward(V).double()
    Pm = gm.forward(V.flip(2).contiguous()).double()
    ef = float((P - Pm[perm].flip(2)).norm() / P.norm())
    y = torch.from_numpy(rng.uniform(na * 256 * 256).reshape(na, 256, 256).astype(np.float32)).to(DEV)
    ym = torch.empty_like(y)
    ym[perm] = y.flip(2)
    D = g.back(y).double()
    Dm = gm.back(ym.contiguous()).double()
    ed = float((D - Dm.flip(2)).norm() / D.norm())
    say("mirror: forward rel-L2 %.3e, deposit rel-L2 %.3e" % (ef, ed))
    assert ef <= 1e-6 and ed <= 1e-6
    gm.close()


def test_c2_full_bitwise_repeatable(c2_full):
    """At the full benchmark size both operators give the same bits on every
    call (integer sums per pixel and per voxel), with FP32 and BF16 data."""
    p, t, g = c2_full
    rng = synth.SplitMix64(29)
    y = torch.from_numpy(rng.uniform(360 * 256 * 256).reshape(360, 256, 256).astype(np.float32)).to(DEV)
    say("c2 full, two calls of each operator")
    for tdt in (torch.float32, torch.bfloat16):
        x = to_dev(t, tdt)
        yy = y.to(tdt)
        assert torch.equal(g.forward(x, out_dtype=tdt), g.forward(x, out_dtype=tdt))
        assert torch.equal(g.back(yy), g.back(yy))


def test_c2_full_adjoint_identity(c2_full):
    p, t, g = c2_full
    rng = synth.SplitMix64(23)
    x = to_dev(t)
    y = torch.from_numpy(rng.uniform(360 * 256 * 256).reshape(360, 256, 256).astype(np.float32)).to(DEV)
    say("c2 full adjoint identity, 360 angles")
    Ax = g.forward(x).double()
    g.set_forward_variant(vam.FWD_RAY)
    Ax_ray = g.forward(x).double()
    g.set_forward_variant(vam.FWD_DEFAULT)
    say("ray-driven forward vs default, rel-L2 %.3e" % float((Ax_ray - Ax).norm() / Ax.norm()))
    assert float((Ax_ray - Ax).norm() / Ax.norm()) <= 2e-6
    lhs = float((Ax * y.double()).sum())
    scale = float(Ax.norm() * y.double().norm())
    res = {}
    for variant in (vam.ADJ_DEFAULT, vam.ADJ_RAY, vam.ADJ_GATHER):
        g.set_adjoint_variant(variant)
        Aty = g.back(y).double()
        rhs = float((x.double() * Aty).sum())
        res[variant] = abs(lhs - rhs) / abs(lhs)
        say("variant %d: <Ax,y> %.12e  <x,A^T y> %.12e  rel %.3e  (vs |Ax||y|: %.3e)"
            % (variant, lhs, rhs, res[variant], abs(lhs - rhs) / scale))
    g.set_adjoint_variant(vam.ADJ_DEFAULT)
    # FP64 accumulation: only the FP32 weights round; the FP32 forward sums
    # (~7000 terms per pixel) bound the agreement
    assert max(res.values()) <= 5e-7


# --------------------------------------------------- optimisation step ----

def test_optimize_step_matches_oracle_loss_and_gradient():
    p = scaled(synth.workload("c1"), n_angles=30)
    t, _ = synth.random_config1_target(64, 32.0, seed=4)
    og = oracle.Geometry(p)
    # start from scaled projections of the target
    P0 = oracle.forward(og, t)
    D0 = oracle.adjoint(og, P0)
    g0 = P0 * (1.0 / np.percentile(D0[t > 0], 50))
    loss_o, dose_o, grad_o = oracle.loss_grad(og, t, g0, 20.0, 0.8)
    g = gpu_geom(p)
    gp = to_dev(g0)
    dose = torch.empty(g.vol_shape, device=DEV)
    lr = 0.5
    loss = g.optimize_step(to_dev(t), gp, threshold=0.8, sharpness=20.0, lr=lr, dose=dose)
    say("loss gpu %.9e oracle %.9e" % (loss, loss_o))
    assert loss == pytest.approx(loss_o, rel=1e-5)
    check(dose.cpu().numpy(), dose_o)
    expect = np.maximum(g0 - lr * grad_o, 0)
    # compare the step actually taken, where the clamp is inactive
    step_g = g0 - gp.double().cpu().numpy()
    step_o = g0 - expect
    free = expect > 0
    e = relL2(step_g[free], step_o[free])
    say("gradient step rel-L2 %.3e" % e)
    assert e <= 1e-4
    g.close()


# ------------------------------------------------- c4: 512^3 precision ----
#
# 512^3, 360 angles, 512^2 DMD, 8 pupil samples, 15 deg edge chief ray.
# Per-projection error against the FP64 oracle of the volume as given (not
# as stored): reduced-precision storage rounds the volume once and each
# projection value once, so for a non-negative volume every projection
# value is within 2u of the oracle's (u = 2^-8 BF16, 2^-11 FP16), plus the
# FP32 accumulation; FP32 storage is held to 1e-5.

C4_FULL = [0, 45, 90, 140, 185, 230, 275, 320]          # full 512^2 projections
C4_ANGLES = [int(k * 360 // 64) for k in range(64)]     # the 64 error angles
U = {"f32": 0.0, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}
TDT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


@pytest.fixture(scope="module")
def c4_case():
    p = synth.workload("c4")
    n = 512
    t, _ = synth.random_config2_target(n, p["r_inner"], seed=0)
    blob = synth.gaussian_blob_volume((n, n, n), (20.0, -35.0, 10.0), 60.0).astype(np.float32)
    vol = 0.6 * t + 0.4 * blob
    og = oracle.Geometry(p)
    say("c4 oracle: %d full projections" % len(C4_FULL))
    full = {a: oracle.forward(og, vol, a0=a, na=1)[0] for a in C4_FULL}
    rng = synth.SplitMix64(40)
    vv = (rng.uniform(64 * 64) * n).astype(np.int32)
    uu = (rng.uniform(64 * 64) * n).astype(np.int32)
    ang = np.repeat(C4_ANGLES, 64).astype(np.int32)
    say("c4 oracle: 64 pixels on each of the 64 error angles")
    sampled = oracle.forward_pixels(og, vol, ang, vv, uu)
    g = gpu_geom(p)
    yield dict(p=p, vol=vol, og=og, full=full, ang=ang, vv=vv, uu=uu, sampled=sampled, g=g)
    g.close()


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16"])
def test_c4_per_projection_error_64_angles(c4_case, dt):
    """Per-projection rel-L2 against the FP64 oracle: in full on 8 of the 64
    error angles, on 64 sampled pixels on every one of them; and each full
    projection's pixels within 2u of their own value plus 1e-5 of the
    projection's largest (FP32: within 1e-5 of the largest)."""
    c = c4_case
    u = U[dt]
    bound = 1e-5 if dt == "f32" else 2 * u
    say("c4 forward", dt)
    P = c["g"].forward(to_dev(c["vol"], TDT[dt]), out_dtype=TDT[dt]).float().cpu().numpy()
    per_full = []
    for a in C4_FULL:
        ref = c["full"][a]
        per_full.append(relL2(P[a], ref))
        err = np.abs(P[a].astype(np.float64) - ref)
        assert np.all(err <= 2.0 * u * np.abs(ref) + 1e-5 * np.abs(ref).max()), (dt, a)
    got = P[c["ang"], c["vv"], c["uu"]]
    per = [relL2(got[i * 64:(i + 1) * 64], c["sampled"][i * 64:(i + 1) * 64]) for i in range(64)]
    say("c4 %s per-projection rel-L2: full projections max %.3e mean %.3e; 64 angles sampled max %.3e "
        "mean %.3e (bound %.3e)" % (dt, max(per_full), np.mean(per_full), max(per), np.mean(per), bound))
    assert max(per_full) <= bound and max(per) <= bound


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_c4_deposit_two_angles(c4_case, dt):
    """Deposit of two full 512^2 projections (U[0,1), stored in FP32 or
    BF16) against the oracle of the values as given: the rounding of each
    stored projection value moves each voxel by at most u of its own dose."""
    c = c4_case
    u = U[dt]
    rng = synth.SplitMix64(44)
    for a in (33, 212):
        y = rng.uniform(512 * 512).reshape(1, 512, 512)
        say("c4 deposit", dt, "angle", a)
        D = c["g"].back(to_dev(y, TDT[dt]), angle_begin=a).cpu().numpy().astype(np.float64)
        ref = oracle.adjoint(c["og"], y, a0=a, na=1)
        e2 = relL2(D, ref)
        em = float((np.abs(D - ref) - u * np.abs(ref)).max() / np.abs(ref).max())
        say("c4 %s deposit angle %d: rel-L2 %.3e, max element error beyond u|ref| %.3e of max"
            % (dt, a, e2, em))
        assert e2 <= (1e-5 if dt == "f32" else 2 * u) and em <= 1e-5
