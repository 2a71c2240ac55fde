"""Whole-path invariants of the reference on generated ligands."""
import numpy as np

import oracle
from paper_1901_06229_amd import synth
from tests.helpers import IDENTITY, np_voxel


def test_score_never_decreases_and_pose_stays_clash_free():
    pocket = synth.pocket(1)
    ligs = synth.ligands(2, count=8)
    orient = synth.orientations(2, 4)
    for l in range(ligs.n_ligands):
        lig = ligs.ligand(l)
        R = len(lig["rot_axis"])
        for o in orient:
            tr = oracle.trace_item(pocket, lig, o, 64)
            for r in range(R):
                assert tr.prof_flags[r, 0] & oracle.FLAG_VALID, "k = 0 (current pose) is valid"
                k = int(tr.k_star[r])
                assert k >= 0
                assert tr.prof_s[r, k] >= tr.prof_s[r, 0]
                if r + 1 < R:  # the next step starts from the chosen pose
                    assert abs(tr.prof_s[r + 1, 0] - tr.prof_s[r, k]) < 1e-9
            if R:
                assert abs(tr.score - tr.prof_s[R - 1, int(tr.k_star[R - 1])]) < 1e-9
            X = tr.xyz
            d = np.linalg.norm(X[:, None] - X[None], axis=-1)
            X0 = lig["xyz"].astype(np.float64)
            d0 = np.linalg.norm(X0[:, None] - X0[None], axis=-1)
            far = d0 > 2.5  # not bonded, not 1-3
            assert (d[far] >= 2.0 - 1e-9).all()


def test_orientation_permutation_and_best():
    pocket = synth.pocket(1)
    ligs = synth.ligands(2, count=5)
    orient = synth.orientations(2, 12)
    a = oracle.dock_batch(pocket, ligs, orient, 32)
    perm = np.random.default_rng(0).permutation(12)
    b = oracle.dock_batch(pocket, ligs, orient[perm], 32)
    assert np.allclose(b.all_scores, a.all_scores[:, perm])
    for l in range(ligs.n_ligands):
        s = a.all_scores[l]
        assert a.best_orient[l] == int(np.argmax(s))  # lowest index on ties
        assert perm[b.best_orient[l]] in np.nonzero(s == s.max())[0]
        assert a.best_score[l] == s.max()


def test_identity_orientation_without_rotamers_is_rigid_score():
    pocket = synth.pocket(1)
    ligs = synth.ligands(2, count=4)
    for l in range(ligs.n_ligands):
        lig = ligs.ligand(l)
        lig0 = dict(xyz=lig["xyz"], rot_axis=np.zeros((0, 2), np.int32),
                    move_offset=np.zeros(1, np.int32), move_atoms=np.zeros(0, np.int16))
        tr = oracle.trace_item(pocket, lig0, IDENTITY, 16)
        X0 = lig["xyz"].astype(np.float64)
        assert np.array_equal(tr.xyz, X0)
        assert tr.score == np_voxel(pocket, X0).sum()
