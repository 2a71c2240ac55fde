"""Pins for the reference's rigid alignment (paper §3.1, first phase; §4.1:
rotation and scoring fused, a reduction to the best orientation, one final
rotation): a planted optimum with the centroid away from the origin (a
rotation applied transposed, or about the origin, picks another candidate),
ties, rigidity invariants, brute force over the candidates with numpy and
scipy, and the equivalence of alignment with the composed rigid transform."""
import numpy as np
from scipy.spatial.transform import Rotation

import oracle
from paper_1901_06229_amd import synth
from tests.helpers import IDENTITY, TinyPocket, apply_orient, make_lig, np_voxel

SHIFT = np.array([3.0, -2.0, 1.5])
# three atoms whose centroid is exactly SHIFT
REL = np.array([[2.1, 0.06, 0.1], [-1.05, 0.47, 0.1], [-1.05, -0.53, -0.2]])


def _rot(axis, deg):
    return Rotation.from_euler(axis, deg, degrees=True).as_matrix().astype(np.float32)


def _hot_box_pocket():
    """Value 1 in the cells whose centres lie in |x|<0.5, 1.5<=y<=2.5, |z|<0.5
    relative to SHIFT, 0 elsewhere; 40^3 cells of 0.25 A around SHIFT."""
    h, G = 0.25, 40
    origin = (SHIFT - 5.0).astype(np.float32)
    c = -5.0 + (np.arange(G) + 0.5) * h
    cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
    hot = (np.abs(cx) < 0.5) & (cy >= 1.5) & (cy <= 2.5) & (np.abs(cz) < 0.5)
    return TinyPocket(hot.astype(np.float32), origin, h)


def _rigid_lig():
    return make_lig(SHIFT + REL, [])


def test_planted_rotation_about_the_centroid():
    p = _hot_box_pocket()
    lig = _rigid_lig()
    rots = np.stack([np.eye(3, dtype=np.float32), _rot("z", -90), _rot("z", 90), _rot("x", 180)])
    tr = oracle.trace_item(p, lig, IDENTITY, 8, align=rots)
    # only +90 degrees about z brings the far atom into the hot box
    assert tr.a_star == 2
    np.testing.assert_array_equal(tr.align_s, [0.0, 0.0, 1.0, 0.0])
    X = lig["xyz"].astype(np.float64)
    c = X.mean(0)
    want = c + (X - c) @ rots[2].astype(np.float64).T
    np.testing.assert_allclose(tr.xyz, want, atol=1e-12)
    assert tr.score == 1.0
    # following another rotation applies that one
    tr1 = oracle.trace_item(p, lig, IDENTITY, 8, align=rots, forced_a=1)
    assert tr1.a_star == 2
    np.testing.assert_allclose(tr1.xyz, c + (X - c) @ rots[1].astype(np.float64).T, atol=1e-12)
    assert tr1.score == 0.0


def test_ties_take_the_lowest_index():
    p = _hot_box_pocket()
    lig = _rigid_lig()
    rots = np.stack([_rot("x", 180), _rot("z", 90), _rot("z", 90), _rot("z", -90)])
    assert oracle.trace_item(p, lig, IDENTITY, 8, align=rots).a_star == 1
    const = TinyPocket(np.full((40, 40, 40), 0.5, np.float32), p.origin, p.spacing)
    tr = oracle.trace_item(const, lig, IDENTITY, 8, align=synth.align_rotations(1, 16)[::-1].copy())
    assert tr.a_star == 0 and (tr.align_s == 1.5).all()


def test_identity_set_equals_no_alignment():
    p = synth.pocket(1)
    ligs = synth.ligands(2, count=3)
    orient = synth.orientations(2, n=4)
    a = oracle.dock_batch(p, ligs, orient, 32)
    b = oracle.dock_batch(p, ligs, orient, 32, align=np.eye(3, dtype=np.float32)[None])
    assert (b.best_align == 0).all() and (b.all_align == 0).all() and (a.best_align == -1).all()
    np.testing.assert_array_equal(a.best_orient, b.best_orient)
    np.testing.assert_array_equal(a.angle_idx, b.angle_idx)
    np.testing.assert_allclose(a.all_scores, b.all_scores, atol=1e-9)
    np.testing.assert_allclose(a.xyz, b.xyz, atol=1e-9)


def test_alignment_is_rigid_and_matches_brute_force():
    p = synth.pocket(1)
    ligs = synth.ligands(2, count=4)
    rots = synth.align_rotations(2, 64)
    R64 = rots.astype(np.float64)
    orient = synth.orientations(2, n=3)
    checked = total = 0
    for l in range(ligs.n_ligands):
        lig = ligs.ligand(l)
        none = np.full(max(1, len(lig["rot_axis"])), -1, np.int16)
        for o in range(len(orient)):
            tr = oracle.trace_item(p, lig, orient[o], 16, align=rots, forced_k=none)
            X = apply_orient(lig["xyz"], orient[o])
            c = X.mean(0)
            # every candidate scored by numpy: the same values except where an
            # atom sits within the ambiguity band of a voxel face
            for a in range(len(rots)):
                s = np_voxel(p, c + (X - c) @ R64[a].T).sum()
                total += 1
                if not tr.align_flags[a] & oracle.FLAG_SAMB:
                    assert abs(s - tr.align_s[a]) <= 1e-9, (l, o, a)
                    checked += 1
                assert tr.align_lo[a] - 1e-9 <= tr.align_s[a] <= tr.align_hi[a] + 1e-9
                assert tr.align_lo[a] - 1e-9 <= s <= tr.align_hi[a] + 1e-9
            assert tr.a_star == int(np.argmax(tr.align_s))
            assert tr.align_s[tr.a_star] >= tr.align_s[0]  # the identity is a candidate
            Y = tr.xyz  # no rotamer moves: the aligned pose itself
            np.testing.assert_allclose(Y, c + (X - c) @ R64[tr.a_star].T, atol=1e-9)
            np.testing.assert_allclose(Y.mean(0), c, atol=1e-9)
            dX = np.linalg.norm(X[:, None] - X[None], axis=-1)
            dY = np.linalg.norm(Y[:, None] - Y[None], axis=-1)
            np.testing.assert_allclose(dY, dX, atol=1e-9)
            assert tr.score == tr.align_s[tr.a_star]
    assert checked >= 0.8 * total, (checked, total)


def test_alignment_then_sweep_equals_the_composed_orientation():
    """Aligning restart o by rotation a and sweeping equals sweeping from the
    single rigid transform (R_a R_o, R_a (t_o - c) + c), composed here."""
    p = synth.pocket(1)
    ligs = synth.ligands(2, count=3)
    rots = synth.align_rotations(2, 32)
    orient = synth.orientations(2, n=2)
    for l in range(ligs.n_ligands):
        lig = ligs.ligand(l)
        for o in range(len(orient)):
            tr = oracle.trace_item(p, lig, orient[o], 64, align=rots)
            a = tr.a_star
            X = apply_orient(lig["xyz"], orient[o])
            c = X.mean(0)
            Ro = orient[o][:9].astype(np.float64).reshape(3, 3)
            Ra = rots[a].astype(np.float64)
            T = np.concatenate([(Ra @ Ro).ravel(), Ra @ (orient[o][9:].astype(np.float64) - c) + c])
            # the composed transform is rounded to FP32 on its way in: follow
            # the aligned run's choices and compare what the sweep computes
            ref = oracle.trace_item(p, lig, T.astype(np.float32), 64, forced_k=tr.k_star)
            np.testing.assert_allclose(ref.xyz, tr.xyz, atol=2e-5)
            assert abs(ref.score - tr.score) <= max(1e-9, tr.score_hi - tr.score_lo)


def test_batch_agrees_with_item_traces():
    p = synth.pocket(1)
    ligs = synth.ligands(2, count=3)
    rots = synth.align_rotations(2, 24)
    orient = synth.orientations(2, n=3)
    res = oracle.dock_batch(p, ligs, orient, 32, align=rots)
    for l in range(ligs.n_ligands):
        for o in range(len(orient)):
            tr = oracle.trace_item(p, ligs.ligand(l), orient[o], 32, align=rots)
            assert res.all_align[l, o] == tr.a_star
            assert res.all_scores[l, o] == tr.score
        assert res.best_align[l] == res.all_align[l, res.best_orient[l]]
