"""The reference with several passes over the rotamers (the paper's
num_repetitions, §3.1): a second pass is the same greedy sweep started from
the pose the first pass left, rotamers in the same order."""
import numpy as np

import oracle
from paper_1901_06229_amd import synth
from tests.helpers import IDENTITY


def _gap(prof_row, valid):
    v = np.sort(prof_row[valid])[::-1]
    return v[0] - v[1] if len(v) > 1 else np.inf


def test_second_pass_is_a_sweep_from_the_first_pass_pose():
    pocket = synth.pocket(1)
    ligs = synth.ligands(2, count=6, first=40)
    orient = synth.orientations(2, 3)
    S = 64
    compared = agreed = 0
    for l in range(ligs.n_ligands):
        lig = ligs.ligand(l)
        R = len(lig["rot_axis"])
        if R == 0:
            continue
        for o in orient:
            two = oracle.trace_item(pocket, lig, o, S, passes=2)
            one = oracle.trace_item(pocket, lig, o, S, passes=1)
            # pass 1 of the two-pass run is the one-pass run
            assert np.array_equal(two.k_star[:R], one.k_star)
            assert np.allclose(two.prof_s[:R], one.prof_s, rtol=0, atol=1e-12)
            # pass 2 from the pass-1 pose (rounded to FP32 as every input pose is)
            again = oracle.trace_item(pocket, dict(lig, xyz=one.xyz.astype(np.float32)), IDENTITY,
                                      S, passes=1)
            for r in range(R):
                valid = (two.prof_flags[R + r] & oracle.FLAG_VALID) != 0
                compared += 1
                if two.k_star[R + r] != again.k_star[r]:
                    # only where the FP32 rounding of the pose can decide
                    assert _gap(two.prof_s[R + r], valid) < 1e-4, (l, r)
                    break  # the paths part here; later steps are not comparable
                agreed += 1
                assert np.allclose(two.prof_s[R + r], again.prof_s[r], rtol=0, atol=1e-4)
    assert agreed >= 0.9 * compared, (agreed, compared)


def test_more_passes_never_lower_the_score():
    pocket = synth.pocket(1)
    ligs = synth.ligands(2, count=6, first=60)
    orient = synth.orientations(2, 4)
    one = oracle.dock_batch(pocket, ligs, orient, 48, passes=1)
    two = oracle.dock_batch(pocket, ligs, orient, 48, passes=2)
    three = oracle.dock_batch(pocket, ligs, orient, 48, passes=3)
    # each step may keep the current pose (k = 0 stays valid), so every
    # restart's score is non-decreasing in the number of passes
    assert (two.all_scores >= one.all_scores - 1e-9).all()
    assert (three.all_scores >= two.all_scores - 1e-9).all()
    assert (two.best_score >= one.best_score - 1e-9).all()
    assert len(three.angle_idx) == 3 * int(ligs.rot_offset[-1])
