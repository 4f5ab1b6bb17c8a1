"""Brute-force second code path for tiny grids -- TEST INFRASTRUCTURE.

Builds the projector as an explicit dense matrix on grids of a few hundred
voxels, by evaluating the tent weight max(0, 1 - |p - c|) per axis of every
ray sample against EVERY voxel centre c (no floor, no cell, no stencil), so
that it shares no sampling or interpolation code with the C++ oracle.

Straight rays (index-matched vial) are generated here from their definition
(a line through the pixel's image point, entering the resin cylinder at the
smaller root of |x_xy| = R).  Refracting geometries take their resin
segments (entry, direction, chord length, weight) from the oracle's ray
records, whose tracing is pinned separately by exact optical invariants.
"""
import math

import numpy as np


def straight_rays(p):
    """Resin segments of the index-matched telecentric geometry:
    list of (u, v, entry, direction, L, weight)."""
    assert p["r_outer"] == p["r_inner"] and p["projector"] == 0
    R = p["r_inner"]
    rays = []
    rho = np.asarray(p["pupil_xy"], dtype=np.float64).reshape(-1, 2)
    for v in range(p["nv"]):
        for u in range(p["nu"]):
            Q = np.array([(u - (p["nu"] - 1) / 2) * p["pitch_u"], 0.0,
                          (v - (p["nv"] - 1) / 2) * p["pitch_v"]])
            for j in range(p["n_pupil"]):
                dx, dz = p["pupil"] * rho[j]
                d = np.array([dx, math.sqrt(1 - dx * dx - dz * dz), dz])
                # |Q_xy + t d_xy|^2 = R^2, smaller root
                a = d[0] ** 2 + d[1] ** 2
                b = 2 * (Q[0] * d[0] + Q[1] * d[1])
                c = Q[0] ** 2 + Q[1] ** 2 - R * R
                disc = b * b - 4 * a * c
                if disc <= 0:
                    continue
                t_in = (-b - math.sqrt(disc)) / (2 * a)
                t_out = (-b + math.sqrt(disc)) / (2 * a)
                rays.append((u, v, Q + t_in * d, d, t_out - t_in,
                             1.0 / p["n_pupil"]))
    return rays


def rays_from_records(p, recs):
    """Resin segments from oracle ray records of shape (nv, nu, np, 26)."""
    out = []
    for v in range(p["nv"]):
        for u in range(p["nu"]):
            for j in range(p["n_pupil"]):
                r = recs[v, u, j]
                if r[23] == 0:
                    continue
                out.append((u, v, r[12:15].copy(), r[15:18].copy(), r[20], r[22]))
    return out


def voxel_centres(p):
    nz, ny, nx = p["nz"], p["ny"], p["nx"]
    z, y, x = np.meshgrid(np.arange(nz) - (nz - 1) / 2, np.arange(ny) - (ny - 1) / 2,
                          np.arange(nx) - (nx - 1) / 2, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def dense_matrix(p, rays, angles):
    """A[(a, v, u), voxel] for the given angles (radians)."""
    C = voxel_centres(p)
    nvox = C.shape[0]
    A = np.zeros((len(angles), p["nv"], p["nu"], nvox))
    ds = p["step"]
    for ai, th in enumerate(angles):
        ct, st = math.cos(th), math.sin(th)
        for (u, v, e, d, L, w) in rays:
            K = int(math.floor(L / ds + 0.5))
            s = (np.arange(K) + 0.5) * ds
            q = e[None, :] + s[:, None] * d[None, :]
            pv = np.stack([ct * q[:, 0] + st * q[:, 1], -st * q[:, 0] + ct * q[:, 1],
                           q[:, 2]], axis=1)
            diff = np.abs(pv[:, None, :] - C[None, :, :])       # (K, nvox, 3)
            tent = np.prod(np.maximum(0.0, 1.0 - diff), axis=2)  # (K, nvox)
            c = w * ds * np.exp(-p["alpha"] * s)
            A[ai, v, u] += c @ tent
    return A.reshape(len(angles) * p["nv"] * p["nu"], nvox)


def continuum_ray_integral(p, vol, e, d, L, w, theta, sub=64):
    """w * integral_0^L exp(-alpha s) I(Rz(-theta)(e + s d)) ds by the
    midpoint rule with step ds/sub, where I is the tent (trilinear)
    interpolant of `vol`, evaluated by brute force against all voxels."""
    C = voxel_centres(p)
    V = np.asarray(vol, dtype=np.float64).ravel()
    h = p["step"] / sub
    n = int(math.floor(L / h))
    s = (np.arange(n) + 0.5) * h
    ct, st = math.cos(theta), math.sin(theta)
    total = 0.0
    for blk in range(0, n, 4096):
        sb = s[blk:blk + 4096]
        q = e[None, :] + sb[:, None] * d[None, :]
        pv = np.stack([ct * q[:, 0] + st * q[:, 1], -st * q[:, 0] + ct * q[:, 1],
                       q[:, 2]], axis=1)
        diff = np.abs(pv[:, None, :] - C[None, :, :])
        tent = np.prod(np.maximum(0.0, 1.0 - diff), axis=2)
        total += float(np.sum(np.exp(-p["alpha"] * sb) * (tent @ V))) * h
    return w * total


def count_samples(p, rays, angles):
    """Samples (over the given angles, radians) whose anti-aliasing stencil
    touches the grid, counted by brute force: a sample counts when its tent
    weight prod(max(0, 1 - |p - c|)) is nonzero for at least one voxel
    centre c of the grid, every centre tried.  (The operator's stencil
    takes the 8 centres around the sample; it touches the grid exactly when
    one of them carries weight, apart from samples lying exactly on a cell
    face one voxel outside the grid, which have probability zero here.)"""
    C = voxel_centres(p)
    ds = p["step"]
    total = 0
    for th in angles:
        ct, st = math.cos(th), math.sin(th)
        for (_u, _v, e, d, L, _w) in rays:
            K = int(math.floor(L / ds + 0.5))
            s = (np.arange(K) + 0.5) * ds
            q = e[None, :] + s[:, None] * d[None, :]
            pv = np.stack([ct * q[:, 0] + st * q[:, 1], -st * q[:, 0] + ct * q[:, 1],
                           q[:, 2]], axis=1)
            tent = np.prod(np.maximum(0.0, 1.0 - np.abs(pv[:, None, :] - C[None, :, :])), axis=2)
            total += int(np.count_nonzero(tent.max(axis=1) > 0.0))
    return total
