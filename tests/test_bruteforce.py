"""Brute force over every angle tuple on tiny ligands (n <= 10, R <= 3, S <= 16)
against the greedy definition (paper §3.1: greedy optimisation of each
fragment in sequence; §4.1: parallel evaluation then a reduction per
fragment).  Poses are built independently with scipy rotations."""
import numpy as np
import pytest

import oracle
from tests.helpers import (IDENTITY, apply_orient, chain_ligand, enumerate_tuples, make_lig,
                           np_voxel, random_pocket, step_pose, step_valid)


def _tiny_ligands():
    X = chain_ligand(9, seed=11)
    X -= X.mean(0)
    yield make_lig(X, [(2, 3, [4, 5, 6, 7, 8])])                                     # R = 1
    yield make_lig(X, [(1, 2, [3, 4, 5, 6, 7, 8]), (4, 5, [6, 7, 8])])                # nested
    yield make_lig(X, [(1, 2, [3, 4, 5, 6, 7, 8]), (3, 4, [5, 6, 7, 8]), (5, 6, [7, 8])])
    X2 = chain_ligand(10, seed=3)
    X2 -= X2.mean(0)
    yield make_lig(X2, [(0, 1, list(range(2, 10))), (6, 7, [8, 9])])


def _greedy_reference(pocket, lig, orient, S, r_bump):
    """Greedy by enumeration: at step r try every k with the earlier choices fixed."""
    X = apply_orient(lig["xyz"], orient)
    ks = []
    for r in range(len(lig["rot_axis"])):
        best, bk, Y_best = None, -1, X
        for k in range(S):
            Y = step_pose(X, lig, r, k, S)
            if not step_valid(X, Y, lig, r, r_bump):
                continue
            s = np_voxel(pocket, Y).sum()
            if best is None or s > best:
                best, bk, Y_best = s, k, Y
        ks.append(bk)
        X = Y_best
    return ks, X


@pytest.mark.parametrize("S", [8, 12, 16])
def test_greedy_step_is_argmax_with_greedy_prefix(S):
    rng = np.random.default_rng(S)
    checked = trials = 0
    for lig in _tiny_ligands():
        for trial in range(3):
            trials += 1
            pocket = random_pocket(rng, G=24, h=0.5)
            # a random sub-voxel shift keeps one geometric near-coincidence of
            # an atom with a face from repeating over every trial
            pocket.origin = (pocket.origin + rng.uniform(0, 0.5, 3)).astype(np.float32)
            orient = IDENTITY
            tr = oracle.trace_item(pocket, lig, orient, S, r_bump=2.0)
            if (tr.prof_flags & (oracle.FLAG_VAMB | oracle.FLAG_SAMB)).any():
                continue  # a face or the radius within 1e-4 A: skip, not a pin
            ks, X = _greedy_reference(pocket, lig, orient, S, 2.0)
            assert list(tr.k_star) == ks
            assert np.abs(tr.xyz - X).max() < 1e-9
            assert abs(tr.score - np_voxel(pocket, X).sum()) < 1e-9
            checked += 1
    # the band is 1e-4 A wide: nearly every trial is a real comparison
    assert checked >= 0.8 * trials, (checked, trials)


@pytest.mark.parametrize("S", [8, 16])
def test_greedy_never_beats_global_max(S):
    rng = np.random.default_rng(100 + S)
    for lig in list(_tiny_ligands())[:3]:
        pocket = random_pocket(rng, G=24, h=0.5)
        tr = oracle.trace_item(pocket, lig, IDENTITY, S, r_bump=2.0)
        tuples = enumerate_tuples(pocket, lig, IDENTITY, S, 2.0)
        feas = [s for _, ok, s in tuples if ok]
        assert tr.score <= max(feas) + 1e-9
        if len(lig["rot_axis"]) == 1:  # R = 1: greedy is exhaustive
            assert abs(tr.score - max(feas)) < 1e-9
        # the greedy tuple itself is feasible and has the reported score
        rec = {t: (ok, s) for t, ok, s in tuples}
        ok, s = rec[tuple(int(k) for k in tr.k_star)]
        assert ok and abs(s - tr.score) < 1e-9


def test_separable_fragments_greedy_is_global_max():
    """Disjoint, non-nested moving sets and no bump test: the score splits into
    one term per rotamer, so greedy reaches the global maximum, and with
    lowest-index tie-breaks the same tuple as lexicographic enumeration."""
    # star: centre 0 with three arms 0-1-2-3, 0-4-5-6, 0-7-8
    d = 1.5
    arms = [np.array([1, 0, 0.0]), np.array([-0.5, 0.866, 0.0]), np.array([-0.5, -0.866, 0.0])]
    xyz = [np.zeros(3)]
    rng = np.random.default_rng(9)
    for arm_i, v in enumerate(arms):
        p = np.zeros(3)
        for s in range(3 if arm_i < 2 else 2):
            w = v + 0.3 * rng.normal(size=3)
            p = p + d * w / np.linalg.norm(w)
            xyz.append(p.copy())
    xyz = np.array(xyz)
    lig = make_lig(xyz, [(1, 2, [3]), (4, 5, [6]), (0, 7, [8])])
    for S in (8, 16):
        for trial in range(4):
            pocket = random_pocket(rng, G=24, h=0.5)
            tr = oracle.trace_item(pocket, lig, IDENTITY, S, r_bump=0.0)
            tuples = enumerate_tuples(pocket, lig, IDENTITY, S, 0.0)
            best = max(s for _, _, s in tuples)
            first = next(t for t, _, s in tuples if s == best)
            assert abs(tr.score - best) < 1e-9
            assert tuple(int(k) for k in tr.k_star) == first
