"""The replay checker's acceptance rule on hand-built step records: which GPU
angle choices it accepts, as what, and which it must refuse."""
from types import SimpleNamespace

import numpy as np

from tests.checker import SAMB, V, VAMB, Report, classify_step


def _tr(ko, scores, flags, lo=None, hi=None):
    sc = np.asarray(scores, np.float64)[None]
    return SimpleNamespace(k_star=np.array([ko]), prof_s=sc,
                           prof_lo=sc.copy() if lo is None else np.asarray(lo, np.float64)[None],
                           prof_hi=sc.copy() if hi is None else np.asarray(hi, np.float64)[None],
                           prof_flags=np.asarray(flags, np.uint8)[None])


def test_same_choice_is_exact():
    assert classify_step(_tr(1, [1, 5, 2], [V, V, V]), 0, 1) == "exact"


def test_tie_within_tolerance():
    tr = _tr(1, [1.0, 5.0, 5.0 - 2e-5], [V, V, V])
    assert classify_step(tr, 0, 2) == "tie"
    tr = _tr(1, [1.0, 5.0, 5.0 - 1e-3], [V, V, V])
    assert classify_step(tr, 0, 2) is None


def test_invalid_angle_refused_unless_near_the_radius():
    tr = _tr(0, [1.0, 9.0], [V, 0])
    assert classify_step(tr, 0, 1) is None
    tr = _tr(0, [1.0, 9.0], [V, VAMB])
    assert classify_step(tr, 0, 1) == "ambiguous"


def test_ambiguous_reference_choice_does_not_excuse_a_worse_angle():
    """The reference's best angle has validity within the band, so the GPU may
    have rejected it; it must then take the best of the rest, not any angle."""
    flags = [V, V | VAMB, V, V]
    scores = [1.0, 9.0, 7.0, 3.0]
    tr = _tr(1, scores, flags)
    assert classify_step(tr, 0, 2) == "ambiguous"   # the best remaining angle
    assert classify_step(tr, 0, 3) is None          # beaten by angle 2
    assert classify_step(tr, 0, 0) is None


def test_score_interval_overlap():
    flags = [V, V | SAMB, V | SAMB]
    scores = [1.0, 5.0, 4.0]
    # angle 2's interval reaches the bottom of angle 1's
    tr = _tr(1, scores, flags, lo=[1.0, 4.5, 3.9], hi=[1.0, 5.1, 4.6])
    assert classify_step(tr, 0, 2) == "ambiguous"
    tr = _tr(1, scores, flags, lo=[1.0, 4.7, 3.9], hi=[1.0, 5.1, 4.6])
    assert classify_step(tr, 0, 2) is None


def test_no_move():
    # the GPU found nothing valid: only acceptable if nothing is clearly valid
    assert classify_step(_tr(0, [1.0, 2.0], [V | VAMB, VAMB]), 0, -1) == "ambiguous"
    assert classify_step(_tr(0, [1.0, 2.0], [V, VAMB]), 0, -1) is None
    # the reference found nothing valid: the GPU's choice must be near the radius
    assert classify_step(_tr(-1, [1.0, 2.0], [0, VAMB]), 0, 1) == "ambiguous"
    assert classify_step(_tr(-1, [1.0, 2.0], [0, VAMB]), 0, 0) is None
    assert classify_step(_tr(0, [1.0, 2.0], [V, 0]), 0, 5) is None


def test_rarity_bound():
    r = Report()
    r.items = 100
    r.steps.update({"exact": 990, "ambiguous": 10})
    r.assert_rare()
    r.steps["ambiguous"] = 30
    try:
        r.assert_rare()
    except AssertionError:
        pass
    else:
        raise AssertionError("30 ambiguous steps in 1020 passed the 1 % bound")
    r.steps["ambiguous"] = 0
    r.score_band = 2
    r.assert_rare()
    r.score_band = 3
    try:
        r.assert_rare()
    except AssertionError:
        pass
    else:
        raise AssertionError("3 band-accepted scores with no flagged item passed")
    # half the items whose final pose sits within the face band may cross it
    r.score_flagged = 20
    r.score_band = 10
    r.assert_rare()
    r.score_band = 11
    try:
        r.assert_rare()
    except AssertionError:
        pass
    else:
        raise AssertionError("11 band-accepted scores of 20 flagged items passed the 1/2 bound")
