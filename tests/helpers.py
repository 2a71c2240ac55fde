"""Independent constructions used to pin the FP64 reference.

Nothing here calls the reference's arithmetic: rotations come from
scipy.spatial.transform (axis-angle -> matrix), voxel lookups from numpy
indexing, and moving / static sets straight from the input arrays.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
from scipy.spatial.transform import Rotation


@dataclass
class TinyPocket:
    grid: np.ndarray     # [nz, ny, nx] float32
    origin: np.ndarray   # [3] float32
    spacing: float


def np_voxel(pocket, pts):
    """Voxel values at points [m,3]: cell floor((p-o)/h), clamped per axis."""
    pts = np.atleast_2d(np.asarray(pts, np.float64))
    nz, ny, nx = pocket.grid.shape
    f = np.floor((pts - pocket.origin.astype(np.float64)) / float(pocket.spacing)).astype(np.int64)
    ix = np.clip(f[:, 0], 0, nx - 1)
    iy = np.clip(f[:, 1], 0, ny - 1)
    iz = np.clip(f[:, 2], 0, nz - 1)
    return pocket.grid[iz, iy, ix].astype(np.float64)


def scipy_rotate(points, a, b, theta):
    """Rotate points by theta about the axis from a to b (right-handed), via scipy."""
    a = np.asarray(a, np.float64)
    u = np.asarray(b, np.float64) - a
    u /= np.linalg.norm(u)
    R = Rotation.from_rotvec(theta * u).as_matrix()
    return (np.asarray(points, np.float64) - a) @ R.T + a


def apply_orient(xyz, orient):
    o = np.asarray(orient, np.float64)
    R = o[:9].reshape(3, 3)
    t = o[9:12]
    return np.asarray(xyz, np.float32).astype(np.float64) @ R.T + t


def cross_sets(lig, r):
    n = len(lig["xyz"])
    mo = lig["move_offset"]
    M = np.asarray(lig["move_atoms"][mo[r]:mo[r + 1]], np.int64)
    a, b = (int(v) for v in lig["rot_axis"][r])
    Q = np.array([j for j in range(n) if j not in set(M.tolist()) and j not in (a, b)], np.int64)
    return a, b, M, Q


def step_pose(X, lig, r, k, S):
    """Pose after rotating rotamer r's moving set by angle step k (scipy)."""
    a, b, M, Q = cross_sets(lig, r)
    Y = X.copy()
    if k != 0 and len(M):
        Y[M] = scipy_rotate(X[M], X[a], X[b], 2 * np.pi * k / S)
    return Y


def step_valid(X, Y, lig, r, r_bump):
    a, b, M, Q = cross_sets(lig, r)
    if len(M) == 0 or len(Q) == 0:
        return True
    d2 = ((Y[M][:, None, :] - X[Q][None, :, :]) ** 2).sum(-1)
    return bool((d2 >= r_bump * r_bump).all())


def enumerate_tuples(pocket, lig, orient, S, r_bump):
    """Every angle tuple: (tuple, feasible along the path, final score, per-step poses)."""
    X0 = apply_orient(lig["xyz"], orient)
    R = len(lig["rot_axis"])
    out = []
    for tup in itertools.product(range(S), repeat=R):
        X = X0
        ok = True
        for r, k in enumerate(tup):
            Y = step_pose(X, lig, r, k, S)
            ok = ok and step_valid(X, Y, lig, r, r_bump)
            X = Y
        out.append((tup, ok, float(np_voxel(pocket, X).sum())))
    return out


def chain_ligand(n, seed=0, jitter=0.0):
    """Zig-zag chain 0-1-2-..., 1.5 A bonds, 109.5 deg angles, random dihedrals."""
    rng = np.random.default_rng(seed)
    pos = [np.zeros(3), np.array([1.5, 0, 0])]
    th = np.deg2rad(109.5)
    for i in range(2, n):
        b = pos[i - 1] - pos[i - 2]
        b /= np.linalg.norm(b)
        w = np.cross(b, [0.3, 0.5, 0.81])
        w /= np.linalg.norm(w)
        phi = rng.uniform(np.deg2rad(60), np.deg2rad(300)) + jitter
        side = np.cos(phi) * w + np.sin(phi) * np.cross(b, w)
        d = -np.cos(th) * b + np.sin(th) * side
        pos.append(pos[i - 1] + 1.5 * d / np.linalg.norm(d))
    return np.array(pos)


def make_lig(xyz, rotamers):
    """rotamers: list of (a, b, moving list)."""
    mo = [0]
    mv = []
    for a, b, M in rotamers:
        mv.extend(sorted(M))
        mo.append(len(mv))
    return dict(xyz=np.asarray(xyz, np.float32),
                rot_axis=np.asarray([(a, b) for a, b, _ in rotamers], np.int32).reshape(-1, 2),
                move_offset=np.asarray(mo, np.int32),
                move_atoms=np.asarray(mv, np.int16))


IDENTITY = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)


def random_pocket(rng, G=24, h=0.5, kind="random"):
    origin = np.full(3, -G * h / 2, np.float32)
    if kind == "random":
        grid = rng.uniform(0.0, 1.0, (G, G, G)).astype(np.float32)
    elif kind == "const":
        grid = np.full((G, G, G), 0.75, np.float32)
    elif kind == "linear_x":
        grid = np.broadcast_to(np.arange(G, dtype=np.float32)[None, None, :], (G, G, G)).copy()
    else:
        raise ValueError(kind)
    return TinyPocket(grid, origin, float(h))
