"""Schedule choice of the autotuner (host logic only)."""
from paper_1208_2407_amd.autotune import TIE, pick


def test_pick_fastest_when_clear():
    timed = [(3.0, (5, 0, 1, 2)), (2.5, (6, 0, 1, 2)), (4.0, (4, 0, 1, 1))]
    assert pick(timed) == (6, 0, 1, 2)


def test_pick_fewest_steps_within_tie():
    # 6 steps per pass is 0.25% faster: a tie, so the shallower schedule is kept
    timed = [(2.863, (5, 0, 1, 2)), (2.856, (6, 0, 1, 2)), (3.19, (4, 0, 1, 1))]
    assert pick(timed) == (5, 0, 1, 2)


def test_pick_tie_prefers_faster_of_same_depth():
    timed = [(2.000, (4, 0, 1, 2)), (1.995, (4, 0, 1, 1)), (1.990, (5, 0, 1, 2))]
    assert pick(timed) == (4, 0, 1, 1)


def test_pick_tie_bound():
    t = 2.0
    assert pick([(t * (1 + TIE) * 1.001, (3, 0, 1, 1)), (t, (4, 0, 1, 1))]) == (4, 0, 1, 1)
    assert pick([(t * (1 + TIE) * 0.999, (3, 0, 1, 1)), (t, (4, 0, 1, 1))]) == (3, 0, 1, 1)


def test_td_candidates_stay_within_the_time_dependent_march():
    from paper_1208_2407_amd.autotune import TD_CANDIDATES
    assert {c[0] for c in TD_CANDIDATES} == {1, 2, 3, 4, 5, 6}
    assert {c[3] for c in TD_CANDIDATES} == {1, 2}
    assert all(c[1] == 0 and c[2] == 1 for c in TD_CANDIDATES)
