"""Pins for the reference's ambiguity band: the voxel-value interval and the
validity flag that the replay checker uses to accept an FP32 choice that
differs from the FP64 one.

A voxel lookup is a step function of the coordinate and the bump test a step
function of the pair distance (paper §4.1: every angle is checked for
validity, then scored); within delta = 1e-4 A of a step the two precisions may
land on different sides.  These tests fix the band by closed forms: which
voxels an atom near a face can reach, the clamped borders, and which pair
distances flag an angle's validity as ambiguous.
"""
import itertools

import numpy as np
import pytest

import oracle
from tests.helpers import IDENTITY, TinyPocket, make_lig, np_voxel, random_pocket

D = oracle.DELTA


def _pocket(seed=0, G=12, h=0.5):
    return random_pocket(np.random.default_rng(seed), G=G, h=h)


def _face(p, axis, i):
    """Coordinate of the face between cells i-1 and i on an axis."""
    return float(p.origin[axis]) + i * p.spacing


def _centre(p, idx):
    return np.asarray(p.origin, np.float64) + (np.asarray(idx, np.float64) + 0.5) * p.spacing


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("side", [-1, 1])
def test_half_band_from_a_face_spans_both_voxels(axis, side):
    p = _pocket(axis)
    g = p.grid
    for i in (3, 6, 9):
        idx = [5, 7, 4]
        pt = _centre(p, idx)
        pt[axis] = _face(p, axis, i) + side * D / 2
        lo_i = list(idx)
        hi_i = list(idx)
        lo_i[axis], hi_i[axis] = i - 1, i
        a = float(g[lo_i[2], lo_i[1], lo_i[0]])
        b = float(g[hi_i[2], hi_i[1], hi_i[0]])
        lo, hi, amb = oracle.voxel_interval(p, pt)
        assert amb
        assert (lo, hi) == (min(a, b), max(a, b))
        # the value itself is the voxel on the point's own side of the face
        assert oracle.voxel_value(p, pt) == (b if side > 0 else a)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("side", [-1, 1])
def test_two_bands_from_a_face_is_one_voxel(axis, side):
    p = _pocket(10 + axis)
    for i in (2, 5, 8):
        pt = _centre(p, [4, 6, 5])
        pt[axis] = _face(p, axis, i) + side * 2 * D
        lo, hi, amb = oracle.voxel_interval(p, pt)
        v = oracle.voxel_value(p, pt)
        assert not amb
        assert lo == hi == v == np_voxel(p, pt)[0]


def test_alternate_voxel_is_on_the_near_side():
    """Only the neighbour across the near face joins the interval: the cell
    across the far face, however extreme its value, stays out."""
    G, h = 12, 0.5
    origin = np.full(3, -G * h / 2, np.float32)
    for axis in range(3):
        grid = np.zeros((G, G, G), np.float32)
        idx = [6, 6, 6]
        up, down = list(idx), list(idx)
        up[axis] += 1
        down[axis] -= 1
        grid[up[2], up[1], up[0]] = 5.0
        grid[down[2], down[1], down[0]] = -5.0
        p = TinyPocket(grid, origin, h)
        pt = _centre(p, idx)
        pt[axis] = _face(p, axis, 7) - D / 2     # in cell 6, near its upper face
        assert oracle.voxel_interval(p, pt) == (0.0, 5.0, True)
        pt[axis] = _face(p, axis, 6) + D / 2     # in cell 6, near its lower face
        assert oracle.voxel_interval(p, pt) == (-5.0, 0.0, True)


def test_corner_reaches_all_eight_cells():
    p = _pocket(21)
    g = p.grid
    for signs in itertools.product((-1, 1), repeat=3):
        c = [5, 6, 7]
        pt = np.array([_face(p, a, c[a]) + signs[a] * D / 3 for a in range(3)])
        cells = [g[c[2] - dz, c[1] - dy, c[0] - dx] for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)]
        lo, hi, amb = oracle.voxel_interval(p, pt)
        assert amb and lo == float(min(cells)) and hi == float(max(cells))
    # near a face on two axes only: the four cells around that edge
    pt = np.array([_face(p, 0, 5) - D / 3, _face(p, 1, 6) + D / 3, _centre(p, [0, 0, 7])[2]])
    cells = [g[7, 6 - dy, 5 - dx] for dx in (0, 1) for dy in (0, 1)]
    lo, hi, amb = oracle.voxel_interval(p, pt)
    assert amb and lo == float(min(cells)) and hi == float(max(cells))


def test_clamped_borders():
    """Outside the box every lookup clamps to the border cell; a face at the
    border has no cell beyond it, so the interval collapses to that cell."""
    p = _pocket(31)
    G = p.grid.shape[0]
    g = p.grid
    for axis in range(3):
        for where, cell in ((-3.0, 0), (_face(p, axis, 0) - D / 2, 0), (_face(p, axis, 0) + D / 2, 0),
                            (_face(p, axis, G) - D / 2, G - 1), (_face(p, axis, G) + D / 2, G - 1),
                            (_face(p, axis, G) + 7.0, G - 1)):
            idx = [4, 5, 6]
            pt = _centre(p, idx)
            if where == -3.0:
                pt[axis] = float(p.origin[axis]) - 3.0
            else:
                pt[axis] = where
            idx[axis] = cell
            v = float(g[idx[2], idx[1], idx[0]])
            lo, hi, _ = oracle.voxel_interval(p, pt)
            assert lo == hi == v == oracle.voxel_value(p, pt)


def test_interval_is_the_range_over_the_band_by_brute_force():
    """For random points, [lo, hi] contains every value reachable by moving
    each coordinate by up to 0.999 delta and nothing beyond the values reachable
    within 1.001 delta (numpy lookups of the 27 shifted points)."""
    rng = np.random.default_rng(5)
    p = _pocket(41, G=10, h=0.25)
    G = p.grid.shape[0]
    shifts = np.array(list(itertools.product((-1.0, 0.0, 1.0), repeat=3)))
    flagged = 0
    for t in range(4000):
        pt = np.asarray(p.origin, np.float64) + rng.uniform(-0.5, G * p.spacing + 0.5, 3)
        if t % 2:
            # snap one axis onto a face, then move it off by up to 2 delta
            a = rng.integers(3)
            i = rng.integers(0, G + 1)
            pt[a] = _face(p, a, i) + rng.uniform(-2 * D, 2 * D)
        lo, hi, amb = oracle.voxel_interval(p, pt)
        inner = np_voxel(p, pt + 0.999 * D * shifts)
        outer = np_voxel(p, pt + 1.001 * D * shifts)
        assert lo <= inner.min() and inner.max() <= hi
        assert outer.min() <= lo and hi <= outer.max()
        frac = (pt - np.asarray(p.origin, np.float64)) / p.spacing
        dist = np.abs(frac - np.round(frac)) * p.spacing
        assert amb == bool((dist < D).any())
        flagged += amb
    assert flagged > 1000


def _pair_ligand(d_list, r_bump=2.0):
    """Axis atoms a = (0,0,-1.5), b = (0,0,0); moving atoms on the +x side at
    z = 1; each static atom placed at distance d from its moving atom, further
    along +x.  Returns the ligand and the distances the FP32 coordinates give."""
    xyz = [[0.0, 0.0, -1.5], [0.0, 0.0, 0.0]]
    moving, static = [], []
    for j, d in enumerate(d_list):
        y = 6.0 * j
        moving.append([1.0, y, 1.0])
        static.append([1.0 + d, y, 1.0])
    xyz = np.array(xyz + moving + static, np.float64)
    m = len(d_list)
    lig = make_lig(xyz, [(0, 1, list(range(2, 2 + m)))])
    X = lig["xyz"].astype(np.float64)
    got = [np.linalg.norm(X[2 + j] - X[2 + m + j]) for j in range(m)]
    return lig, got


@pytest.mark.parametrize("e,valid,vamb", [(D / 2, True, True), (-D / 2, False, True),
                                          (2 * D, True, False), (-2 * D, False, False),
                                          (0.0, True, True)])
def test_validity_flag_at_the_bump_radius(e, valid, vamb):
    rb = 2.0
    lig, got = _pair_ligand([rb + e])
    assert abs(got[0] - (rb + e)) < 1e-6
    p = _pocket(50, G=40, h=0.5)
    tr = oracle.trace_item(p, lig, IDENTITY, 1, r_bump=rb)  # S = 1: only the identity
    f = int(tr.prof_flags[0, 0])
    assert bool(f & oracle.FLAG_VALID) == valid
    assert bool(f & oracle.FLAG_VAMB) == vamb


@pytest.mark.parametrize("ds,valid,vamb", [
    ((-1e-4 / 2, -2e-4), False, False),   # one clash inside the band, one clearly a clash
    ((-1e-4 / 2, -1e-4 / 3), False, True),  # every clash inside the band
    ((1e-4 / 2, 1.5), True, True),        # valid, one pair inside the band
    ((2e-4, 1.5), True, False),           # valid, every pair clear of the band
])
def test_validity_flag_over_several_pairs(ds, valid, vamb):
    rb = 2.0
    lig, got = _pair_ligand([rb + d for d in ds])
    for g_, d in zip(got, ds):
        assert abs(g_ - (rb + d)) < 1e-6
    p = _pocket(51, G=40, h=0.5)
    tr = oracle.trace_item(p, lig, IDENTITY, 1, r_bump=rb)
    f = int(tr.prof_flags[0, 0])
    assert bool(f & oracle.FLAG_VALID) == valid
    assert bool(f & oracle.FLAG_VAMB) == vamb
