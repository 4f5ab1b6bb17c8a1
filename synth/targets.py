"""Seeded binary targets, FP32 {0, 1} arrays of shape (nz, ny, nx) (x fastest).

A voxel is set when its centre lies inside any primitive.  Voxel (i, j, k)
has its centre at (i - (nx-1)/2, j - (ny-1)/2, k - (nz-1)/2) in voxel units,
the vial axis along +z through the origin.  These stand in for the paper's
STL parts, which are not available: unions of spheres, z-cylinders, boxes,
tori and struts, plus the paper's fin stack as a procedural shape.
"""
import numpy as np
from .rng import SplitMix64


def _centres(shape):
    nz, ny, nx = shape
    z = np.arange(nz) - (nz - 1) / 2.0
    y = np.arange(ny) - (ny - 1) / 2.0
    x = np.arange(nx) - (nx - 1) / 2.0
    return z[:, None, None], y[None, :, None], x[None, None, :]


def _inside(prim, z, y, x):
    kind = prim["kind"]
    c = prim["centre"]
    dx, dy, dz = x - c[0], y - c[1], z - c[2]
    if kind == "sphere":
        return dx * dx + dy * dy + dz * dz <= prim["r"] ** 2
    if kind == "zcyl":
        return (dx * dx + dy * dy <= prim["r"] ** 2) & (np.abs(dz) <= prim["h"])
    R = prim.get("rot", np.eye(3))
    # local coordinates l = R^T (p - c)
    lx = R[0, 0] * dx + R[1, 0] * dy + R[2, 0] * dz
    ly = R[0, 1] * dx + R[1, 1] * dy + R[2, 1] * dz
    lz = R[0, 2] * dx + R[1, 2] * dy + R[2, 2] * dz
    if kind == "box":
        h = prim["half"]
        return (np.abs(lx) <= h[0]) & (np.abs(ly) <= h[1]) & (np.abs(lz) <= h[2])
    if kind == "torus":
        rho = np.sqrt(lx * lx + ly * ly)
        return (rho - prim["R"]) ** 2 + lz * lz <= prim["r"] ** 2
    if kind == "strut":
        # capsule along local z with half length h and radius r
        h = prim["h"]
        cz = np.clip(lz, -h, h)
        return lx * lx + ly * ly + (lz - cz) ** 2 <= prim["r"] ** 2
    raise ValueError(kind)


def _extent(p):
    """Radius of a sphere around the centre that holds the primitive."""
    k = p["kind"]
    if k == "zcyl":
        return float(np.hypot(p["r"], p["h"]))
    if k == "gauss":
        return np.inf
    return _bounding_radius(p)


def primitive_target(shape, prims):
    """Union of primitives voxelised at voxel centres, float32 {0,1}.  Each
    primitive is evaluated on the sub-grid of its bounding box only."""
    nz, ny, nx = shape
    z, y, x = _centres(shape)
    out = np.zeros(shape, dtype=bool)
    for p in prims:
        r = _extent(p) + 1.0
        c = p["centre"]
        sl = []
        for ax, (n, ci) in enumerate(((nz, c[2]), (ny, c[1]), (nx, c[0]))):
            lo = max(int(np.floor(ci - r + (n - 1) / 2.0)), 0)
            hi = min(int(np.ceil(ci + r + (n - 1) / 2.0)) + 1, n)
            sl.append(slice(lo, max(lo, hi)))
        zs, ys, xs = z[sl[0]], y[:, sl[1]], x[:, :, sl[2]]
        sub = out[sl[0], sl[1], sl[2]]
        sub |= np.broadcast_to(_inside(p, zs, ys, xs), sub.shape)
    return out.astype(np.float32)


def gaussian_blob_volume(shape, centre, sigma):
    """exp(-|x - c|^2 / (2 sigma^2)) sampled at voxel centres (float64)."""
    z, y, x = _centres(shape)
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return np.exp(-r2 / (2.0 * sigma * sigma))


def _bounding_radius(p):
    k = p["kind"]
    if k == "sphere":
        return p["r"]
    if k == "box":
        return float(np.linalg.norm(p["half"]))
    if k == "torus":
        return p["R"] + p["r"]
    if k == "strut":
        return p["h"] + p["r"]
    raise ValueError(k)


def _place(rng, radius, r_inner, half_z, margin=2.0):
    """Centre whose bounding sphere stays `margin` inside the vial radius
    and the grid's z range."""
    lim_xy = max(r_inner - radius - margin, 0.0)
    lim_z = max(half_z - radius - margin, 0.0)
    while True:
        x, y = rng.uniform(2, -lim_xy, lim_xy)
        if x * x + y * y <= lim_xy * lim_xy:
            break
    z = rng.uniform(None, -lim_z, lim_z)
    return np.array([x, y, z])


def random_config1_target(n, r_inner, seed):
    """Union of 1-3 spheres / z-cylinders, radius U[3, 20], each fully
    inside the vial radius with a 2-voxel margin."""
    rng = SplitMix64(seed)
    prims = []
    for _ in range(rng.integer(1, 3)):
        r = rng.uniform(None, 3.0, 20.0)
        r = min(r, r_inner - 3.0)
        if rng.uniform() < 0.5:
            c = _place(rng, r, r_inner, n / 2.0)
            prims.append({"kind": "sphere", "centre": c, "r": r})
        else:
            h = rng.uniform(None, 3.0, 20.0)
            lim_xy = max(r_inner - r - 2.0, 0.0)
            while True:
                x, y = rng.uniform(2, -lim_xy, lim_xy)
                if x * x + y * y <= lim_xy * lim_xy:
                    break
            zc = rng.uniform(None, -(n / 2.0 - h - 2.0), n / 2.0 - h - 2.0)
            prims.append({"kind": "zcyl", "centre": np.array([x, y, zc]),
                          "r": r, "h": h})
    return primitive_target((n, n, n), prims), prims


def _random_prims(rng, count, kinds, r_inner, half_z):
    prims = []
    for _ in range(count):
        kind = kinds[rng.integer(0, len(kinds) - 1)]
        if kind == "sphere":
            p = {"kind": "sphere", "r": rng.uniform(None, 4.0, 30.0)}
        elif kind == "box":
            p = {"kind": "box", "half": rng.uniform(3, 4.0, 30.0),
                 "rot": rng.rotation()}
        elif kind == "torus":
            p = {"kind": "torus", "R": rng.uniform(None, 8.0, 30.0),
                 "r": rng.uniform(None, 2.0, 6.0), "rot": rng.rotation()}
        else:  # strut: 2-4 voxels wide
            p = {"kind": "strut", "r": 0.5 * rng.uniform(None, 2.0, 4.0),
                 "h": rng.uniform(None, 10.0, 60.0), "rot": rng.rotation()}
        p["centre"] = _place(rng, _bounding_radius(p), r_inner, half_z)
        prims.append(p)
    return prims


def random_config2_target(n, r_inner, seed):
    """5-20 spheres / boxes / tori with random orientation."""
    rng = SplitMix64(seed)
    prims = _random_prims(rng, rng.integer(5, 20), ("sphere", "box", "torus"),
                          r_inner, n / 2.0)
    return primitive_target((n, n, n), prims), prims


def random_config3_target(n, r_inner, seed):
    """Mixtures of spheres, boxes and thin struts 2-4 voxels wide."""
    rng = SplitMix64(seed)
    prims = _random_prims(rng, rng.integer(5, 20), ("sphere", "box", "strut"),
                          r_inner, n / 2.0)
    return primitive_target((n, n, n), prims), prims


def fin_stack_target(n, voxel_mm, fins=9, thickness_mm=1.0, period_mm=2.25,
                     width_mm=8.0, base_mm=2.0):
    """Stack of `fins` parallel plates normal to the vial axis (thickness and
    period as printed in the paper's results section) on a square base,
    joined by a central spine, centred on the axis and in z."""
    z, y, x = _centres((n, n, n))
    half_w = 0.5 * width_mm / voxel_mm
    in_xy = (np.abs(x) <= half_w) & (np.abs(y) <= half_w)
    height = base_mm + fins * period_mm
    zz = z * voxel_mm + 0.5 * height - base_mm   # base occupies [-base_mm, 0)
    base = (zz >= -base_mm) & (zz < 0)
    fin = np.zeros_like(zz, dtype=bool)
    for f in range(fins):
        z0 = f * period_mm + (period_mm - thickness_mm)
        fin |= (zz >= z0) & (zz < z0 + thickness_mm)
    spine = (np.abs(x) <= 0.5 / voxel_mm) & (zz >= 0) & (zz < fins * period_mm)
    vol = (in_xy & (base | fin)) | (spine & (np.abs(y) <= half_w))
    return vol.astype(np.float32)
