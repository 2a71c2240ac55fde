"""FP64 reference of the learned proposal's inputs and targets -- TEST
INFRASTRUCTURE ONLY.

Features of a rotamer step (the network input, 64 values): the grid values on
a 4 x 4 x 4 lattice in the rotamer's local frame -- z along the bond axis
u = (X_b - X_a)/|X_b - X_a| through X_a, x from the axis towards the centroid
of the moving atoms' radial vectors, y = z cross x -- spanning the swept
cylinder: x, y in {-rho, -rho/3, rho/3, rho} with rho the largest radial
distance of a moving atom (at least 1e-3 A), z evenly over
[min z_i - 1, max z_i + 1].  Each value is the voxel value of the lattice
point, clamped below at -1.  Feature index = 16 ix + 4 iy + iz.

Target of a step (the network output, 256 values): the score landscape over
every angle step (valid or not), max(s_k - max_k' s_k', -4).
"""
from __future__ import annotations

import numpy as np


def voxel(pocket, pts):
    pts = np.atleast_2d(np.asarray(pts, np.float64))
    nz, ny, nx = pocket.grid.shape
    f = np.floor((pts - np.asarray(pocket.origin, np.float64)) / float(pocket.spacing))
    ix = np.clip(f[:, 0], 0, nx - 1).astype(np.int64)
    iy = np.clip(f[:, 1], 0, ny - 1).astype(np.int64)
    iz = np.clip(f[:, 2], 0, nz - 1).astype(np.int64)
    return pocket.grid[iz, iy, ix].astype(np.float64)


def lattice_points(X, lig, r):
    """The 64 lattice points (FP64) of rotamer step r for pose X [n, 3]."""
    X = np.asarray(X, np.float64)
    a, b = (int(v) for v in lig["rot_axis"][r])
    mo = lig["move_offset"]
    M = np.asarray(lig["move_atoms"][mo[r]:mo[r + 1]], np.int64)
    u = X[b] - X[a]
    u = u / np.linalg.norm(u)
    v = X[M] - X[a]
    z = v @ u
    rad = v - np.outer(z, u)
    rho = max(float(np.linalg.norm(rad, axis=1).max()) if len(M) else 0.0, 1e-3)
    c = rad.sum(0) if len(M) else np.zeros(3)
    if not (c @ c > 1e-12):
        c = np.cross(u, [1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.cross(u, [0.0, 1.0, 0.0])
    ex = c / np.linalg.norm(c)
    ey = np.cross(u, ex)
    zlo, zhi = (float(z.min()) - 1.0, float(z.max()) + 1.0) if len(M) else (-1.0, 1.0)
    pts = []
    for ix in range(4):
        for iy in range(4):
            for iz in range(4):
                lx = -rho + 2.0 * rho * ix / 3.0
                ly = -rho + 2.0 * rho * iy / 3.0
                lz = zlo + (zhi - zlo) * iz / 3.0
                pts.append(X[a] + lx * ex + ly * ey + lz * u)
    return np.array(pts)


def features(pocket, X, lig, r):
    return np.maximum(voxel(pocket, lattice_points(X, lig, r)), -1.0)


def landscape(profile_scores):
    s = np.asarray(profile_scores, np.float64)
    return np.maximum(s - s.max(axis=-1, keepdims=True), -4.0)
