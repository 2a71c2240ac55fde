"""Pins for the FP64 reference of the learned proposal's inputs and targets
(oracle/features.py): closed-form properties of the score landscape, the
geometry of the 4 x 4 x 4 local-frame lattice, and voxel indexing checked on
constant and linear grids."""
import numpy as np

from oracle.features import features, landscape, lattice_points, voxel
from paper_1901_06229_amd import synth


class _Pocket:
    def __init__(self, grid, origin, spacing):
        self.grid = np.asarray(grid, np.float32)
        self.origin = np.asarray(origin, np.float64)
        self.spacing = float(spacing)


def _ligand(seed=0):
    lig = synth.ligands(1, count=1, first=seed).ligand(0)
    return lig, lig["xyz"].astype(np.float64)


def test_landscape_closed_form():
    s = np.array([3.0, 1.0, -2.0, 3.0, 2.5])
    np.testing.assert_array_equal(landscape(s), [0.0, -2.0, -4.0, 0.0, -0.5])
    rng = np.random.default_rng(0)
    p = rng.normal(scale=5.0, size=(7, 256))
    t = landscape(p)
    assert (t.max(axis=1) == 0.0).all() and (t >= -4.0).all()
    np.testing.assert_allclose(landscape(p + 17.0), t, atol=1e-12)  # shift invariant
    i = p.argmax(axis=1)
    assert (t[np.arange(7), i] == 0.0).all()


def test_lattice_spans_the_swept_cylinder_in_the_bond_frame():
    lig, X = _ligand(3)
    for r in range(len(lig["rot_axis"])):
        a, b = (int(v) for v in lig["rot_axis"][r])
        mo = lig["move_offset"]
        M = np.asarray(lig["move_atoms"][mo[r]:mo[r + 1]], np.int64)
        pts = lattice_points(X, lig, r)
        assert pts.shape == (64, 3)
        u = (X[b] - X[a]) / np.linalg.norm(X[b] - X[a])
        v = X[M] - X[a]
        z = v @ u
        rad = v - np.outer(z, u)
        rho = max(np.linalg.norm(rad, axis=1).max(), 1e-3)
        L = (pts - X[a]).reshape(4, 4, 4, 3)  # [ix][iy][iz]
        # axial coordinates: evenly spaced over [min z - 1, max z + 1], the same for every ix, iy
        ax = L @ u
        np.testing.assert_allclose(ax[0, 0], np.linspace(z.min() - 1.0, z.max() + 1.0, 4), atol=1e-9)
        np.testing.assert_allclose(ax, np.broadcast_to(ax[0, 0], (4, 4, 4)), atol=1e-9)
        # radial part: a square grid of side 2 rho centred on the axis
        radial = L - ax[..., None] * u
        ex = (radial[3, 0, 0] - radial[0, 0, 0]) / (2 * rho)
        ey = (radial[0, 3, 0] - radial[0, 0, 0]) / (2 * rho)
        np.testing.assert_allclose([ex @ ex, ey @ ey, ex @ ey, ex @ u, ey @ u], [1, 1, 0, 0, 0], atol=1e-9)
        np.testing.assert_allclose(np.cross(u, ex), ey, atol=1e-9)  # right-handed frame
        np.testing.assert_allclose(radial[1, 2, 0], (-rho / 3) * ex + (rho / 3) * ey, atol=1e-9)
        if np.linalg.norm(rad.sum(0)) > 1e-6:  # x points to the moving atoms' radial centroid
            assert rad.sum(0) @ ex > 0


def test_features_on_constant_and_linear_grids():
    lig, X = _ligand(5)
    n = 64
    const = _Pocket(np.full((n, n, n), 0.75), [-16.0, -16.0, -16.0], 0.5)
    low = _Pocket(np.full((n, n, n), -9.0), [-16.0, -16.0, -16.0], 0.5)
    # linear grid V = i_x: the feature is floor((x - o_x) / h) clamped to the box (and at -1)
    ix = np.broadcast_to(np.arange(n, dtype=np.float32)[None, None, :], (n, n, n))
    lin = _Pocket(ix, [-16.0, -16.0, -16.0], 0.5)
    for r in range(len(lig["rot_axis"])):
        np.testing.assert_array_equal(features(const, X, lig, r), np.full(64, 0.75))
        np.testing.assert_array_equal(features(low, X, lig, r), np.full(64, -1.0))  # clamped
        pts = lattice_points(X, lig, r)
        want = np.clip(np.floor((pts[:, 0] + 16.0) / 0.5), 0, n - 1)
        np.testing.assert_array_equal(features(lin, X, lig, r), want)


def test_voxel_lookup_centres_and_clamping():
    rng = np.random.default_rng(2)
    g = rng.normal(size=(6, 5, 4)).astype(np.float32)  # [z][y][x]
    p = _Pocket(g, [1.0, -2.0, 0.5], 0.25)
    for (z, y, x) in ((0, 0, 0), (5, 4, 3), (2, 1, 3), (4, 3, 0)):
        c = np.array([1.0 + (x + 0.5) * 0.25, -2.0 + (y + 0.5) * 0.25, 0.5 + (z + 0.5) * 0.25])
        assert voxel(p, c)[0] == np.float64(g[z, y, x])
    # far outside on every axis: the corner voxels
    assert voxel(p, [-50.0, -50.0, -50.0])[0] == np.float64(g[0, 0, 0])
    assert voxel(p, [50.0, 50.0, 50.0])[0] == np.float64(g[5, 4, 3])
