"""Pins for the reference's scoring (grid voxel sum) and bump test, by closed
forms: voxel centres, constant and linear grids, a single hot voxel, and the
cylindrical distance law of a rotating pair."""
import numpy as np

import oracle
from tests.helpers import (IDENTITY, TinyPocket, chain_ligand, make_lig, np_voxel,
                           random_pocket, scipy_rotate)


def test_voxel_centres_return_grid_values():
    rng = np.random.default_rng(0)
    p = random_pocket(rng, G=12, h=0.5)
    for _ in range(300):
        i = rng.integers(0, 12, 3)
        c = p.origin + (i + 0.5) * p.spacing
        assert oracle.voxel_value(p, c) == p.grid[i[2], i[1], i[0]]
    # outside the box: clamped to the border cell
    assert oracle.voxel_value(p, [100.0, -100.0, 0.1]) == p.grid[6, 0, 11]


def _lig8():
    X = chain_ligand(8, seed=5)
    X = X - X.mean(0)
    return make_lig(X, [(1, 2, [3, 4, 5, 6, 7]), (3, 4, [5, 6, 7]), (4, 5, [6, 7])])


def test_constant_grid_all_ties_no_move():
    p = random_pocket(np.random.default_rng(1), G=40, h=0.5, kind="const")
    lig = _lig8()
    tr = oracle.trace_item(p, lig, IDENTITY, 32)
    n = len(lig["xyz"])
    assert np.all(tr.prof_s == n * 0.75)
    assert np.all(tr.k_star == 0)
    assert np.abs(tr.xyz - lig["xyz"].astype(np.float64)).max() == 0.0


def test_linear_grid_closed_form():
    """V = i_x: each angle's score is sum_i clamp(floor((x_i - o)/h)), with the
    rotated coordinates built independently (scipy)."""
    p = random_pocket(np.random.default_rng(2), G=40, h=0.5, kind="linear_x")
    lig = _lig8()
    S = 48
    tr = oracle.trace_item(p, lig, IDENTITY, S, r_bump=0.0)
    X = lig["xyz"].astype(np.float64)
    checked = 0
    for r in range(len(lig["rot_axis"])):
        a, b = lig["rot_axis"][r]
        M = lig["move_atoms"][lig["move_offset"][r]:lig["move_offset"][r + 1]]
        for k in range(S):
            Y = X.copy()
            if k:
                Y[M] = scipy_rotate(X[M], X[a], X[b], 2 * np.pi * k / S)
            ix = np.clip(np.floor((Y[:, 0] - p.origin[0]) / p.spacing), 0, 39)
            if not tr.prof_flags[r, k] & oracle.FLAG_SAMB:
                assert tr.prof_s[r, k] == ix.sum()
                checked += 1
            else:
                assert tr.prof_lo[r, k] <= ix.sum() <= tr.prof_hi[r, k]
        k = int(tr.k_star[r])
        if k:
            X[M] = scipy_rotate(X[M], X[a], X[b], 2 * np.pi * k / S)
    assert checked >= 0.95 * len(lig["rot_axis"]) * S, checked


def test_single_hot_voxel_hitting_angle():
    """One moving atom circling the z axis; only one voxel is hot.  The chosen
    angle is the first step whose point lands in that voxel."""
    G, h = 64, 0.1
    origin = np.full(3, -G * h / 2, np.float32)
    grid = np.zeros((G, G, G), np.float32)
    rho, z0, S = 2.0, 0.375, 90
    kstar = 31
    th = 2 * np.pi * kstar / S
    hot = np.array([rho * np.cos(th), rho * np.sin(th), z0])
    i = np.floor((hot - origin) / h).astype(int)
    grid[i[2], i[1], i[0]] = 1.0
    p = TinyPocket(grid, origin, h)
    # axis atoms a = (0,0,-1.5), b = (0,0,0); moving atom at (rho, 0, z0); a far static atom
    xyz = np.array([[0, 0, -1.5], [0, 0, 0], [rho, 0, z0], [0.0, -2.9, -2.6]])
    lig = make_lig(xyz, [(0, 1, [2])])
    tr = oracle.trace_item(p, lig, IDENTITY, S, r_bump=0.5)
    pts = np.stack([[rho * np.cos(2 * np.pi * k / S), rho * np.sin(2 * np.pi * k / S), z0]
                    for k in range(S)])
    hits = np.nonzero(np_voxel(p, pts) == 1.0)[0]
    assert hits.min() == kstar
    assert tr.k_star[0] == hits.min()
    assert np.abs(tr.xyz[2] - pts[kstar]).max() < 1e-12


def test_bump_matches_cylindrical_closed_form():
    """d^2(theta) = rho_i^2 + rho_j^2 - 2 rho_i rho_j cos(phi_i + theta - phi_j) + (z_i - z_j)^2
    for a moving atom i and a static atom j about the z axis."""
    rng = np.random.default_rng(7)
    p = random_pocket(rng, G=32, h=0.5)
    S = 120
    checked = 0
    for trial in range(40):
        # axis a=(0,0,-1.5) -> b=(0,0,0); moving atoms at z>0, static atoms around
        mv = [[rng.uniform(1.0, 3.0) * np.cos(t), rng.uniform(1.0, 3.0) * np.sin(t), rng.uniform(0.5, 2.0)]
              for t in rng.uniform(0, 2 * np.pi, 2)]
        st = [[rng.uniform(0.5, 3.5) * np.cos(t), rng.uniform(0.5, 3.5) * np.sin(t), rng.uniform(-0.5, 2.5)]
              for t in rng.uniform(0, 2 * np.pi, 2)]
        xyz = np.array([[0, 0, -1.5], [0, 0, 0]] + mv + st)
        lig = make_lig(xyz, [(0, 1, [2, 3])])
        rb = float(rng.uniform(1.0, 2.5))
        tr = oracle.trace_item(p, lig, IDENTITY, S, r_bump=rb)
        X = lig["xyz"].astype(np.float64)
        rho = np.hypot(X[:, 0], X[:, 1])
        phi = np.arctan2(X[:, 1], X[:, 0])
        theta = 2 * np.pi * np.arange(S) / S
        ok = np.ones(S, bool)
        for i in (2, 3):
            for j in (4, 5):
                d2 = (rho[i] ** 2 + rho[j] ** 2 - 2 * rho[i] * rho[j] * np.cos(phi[i] + theta - phi[j])
                      + (X[i, 2] - X[j, 2]) ** 2)
                ok &= d2 >= rb * rb
        valid = (tr.prof_flags[0] & oracle.FLAG_VALID) > 0
        amb = (tr.prof_flags[0] & oracle.FLAG_VAMB) > 0
        assert np.array_equal(valid[~amb], ok[~amb])
        checked += int((~amb).sum())
    assert checked > 40 * S * 0.9
