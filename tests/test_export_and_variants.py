"""NEXT-4 pieces on the CPU: the 8-bit export definition (closed-form
statistics of a ramp, rounding, clipping), the 13-point hexagonal pupil
table and the procedural fin-stack target."""
import math

import numpy as np
import pytest

from oracle import export
import synth


def test_export_statistics_of_a_ramp_are_closed_form():
    n = 1001
    x = np.arange(n, dtype=np.float64)
    mean, sd, clip = export.export_stats(x)
    assert mean == pytest.approx((n - 1) / 2, rel=1e-15)
    assert sd == pytest.approx(math.sqrt((n * n - 1) / 12.0), rel=1e-13)
    assert clip == pytest.approx(mean + 3 * sd, rel=1e-15)


def test_export_levels():
    # clip = mean + 3 sd; values above the clip saturate, negatives map to 0
    x = np.concatenate([np.zeros(996), [1.0, 2.0, 3.0, 1e6]])
    q, (mean, sd, clip) = export.equalize_u8(x)
    assert q[-1] == 255 and q[0] == 0
    assert np.all(np.diff(q[996:]) >= 0)
    # round half to even at exactly half a level
    q2, _ = export.equalize_u8(np.array([0.5, 1.5, 2.5]) * (4.0 / 255.0), stats=(0.0, 0.0, 4.0))
    assert list(q2) == [0, 2, 2]
    q3, _ = export.equalize_u8(np.array([-1.0, 2.0, 4.0, 9.0]), stats=(0.0, 0.0, 4.0))
    assert list(q3) == [0, 128, 255, 255]


def test_hex13_pupil_is_hexagonally_symmetric():
    p = synth.pupil_hex13()
    assert p.shape == (13, 2)
    assert np.all(np.hypot(p[:, 0], p[:, 1]) <= 1 + 1e-12)
    np.testing.assert_allclose(p.mean(axis=0), 0.0, atol=1e-15)
    c, s = math.cos(math.pi / 3), math.sin(math.pi / 3)
    rot = p @ np.array([[c, s], [-s, c]])
    for q in rot:
        assert np.min(np.hypot(*(p - q).T)) < 1e-12
    # centre + inner ring + outer ring
    r = np.sort(np.hypot(p[:, 0], p[:, 1]))
    np.testing.assert_allclose(r, [0] + [0.5] * 6 + [1.0] * 6, atol=1e-15)


def test_fin_stack_has_nine_fins_of_the_printed_period():
    # fin part of the results section: 9 fins, 1 mm thick, 2.25 mm period
    voxel = 0.108
    n = 256
    t = synth.fin_stack_target(n, voxel)
    # a column off the spine, through the fins
    col = t[:, n // 2 + 20, n // 2 + 25] > 0
    rises = np.flatnonzero(np.diff(col.astype(int)) == 1) + 1
    # base + 9 fins, each run about 1 mm (fins) thick
    assert len(rises) == 10
    zs = (np.arange(n) - (n - 1) / 2) * voxel
    np.testing.assert_allclose(np.diff(zs[rises[1:]]), 2.25, atol=voxel)
    falls = np.flatnonzero(np.diff(col.astype(int)) == -1) + 1
    np.testing.assert_allclose((falls[1:] - rises[1:]) * voxel, 1.0, atol=1.01 * voxel)


def test_turned_voxel_support_fits_a_4x4x3_block_of_lab_cells():
    # The fixed-point deposit bounds a voxel's sum by the samples in any
    # 4 x 4 x 3 block of lab-frame unit cells: the voxel's support (open
    # cube of half-width 1 in the volume frame) turned by any angle about z
    # must overlap at most 4 unit cells along lab x and y and 3 along z.
    import math
    rng = synth.SplitMix64(90)
    for _ in range(20000):
        th = rng.uniform() * 2 * math.pi
        c, s = math.cos(th), math.sin(th)
        vx, vy, vz = (rng.uniform(3) - 0.5) * 200.0
        # lab position of the voxel centre and the extent of the turned square
        qx, qy = c * vx - s * vy, s * vx + c * vy
        h = abs(c) + abs(s)
        # unit cells overlapping the open intervals (q - h, q + h), (vz - 1, vz + 1)
        def cells(lo, hi):
            return math.ceil(hi) - math.floor(lo)
        assert cells(qx - h, qx + h) <= 4 and cells(qy - h, qy + h) <= 4
        assert cells(vz - 1.0, vz + 1.0) <= 3
        # the corners of the turned square are within the bounding box
        for dx, dy in ((-1, -1), (-1, 1), (1, -1), (1, 1)):
            lx, ly = c * (vx + dx) - s * (vy + dy), s * (vx + dx) + c * (vy + dy)
            assert qx - h - 1e-9 <= lx <= qx + h + 1e-9 and qy - h - 1e-9 <= ly <= qy + h + 1e-9
