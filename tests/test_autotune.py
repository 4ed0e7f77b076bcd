"""Host logic of the plan autotuner (no GPU): the selection rule."""
from paper_2010_14258_amd import autotune as AT


def test_pick_prefers_fewest_steps_within_tolerance():
    table = [([20, 1, 7, 1], 0.3480), ([10, 1, 7, 1], 0.3500), ([5, 1, 7, 1], 0.3700), ([10, 2, 9, 1], 0.3490)]
    # 0.350 and 0.349 are within 2% of 0.348: the fewest steps per pass wins, then the fewest chunks
    assert AT.pick(table, within=0.02)[0] == [10, 1, 7, 1]
    # a strict tolerance keeps the fastest
    assert AT.pick(table, within=0.0)[0] == [20, 1, 7, 1]
    # the default half-percent margin: 0.3490 is within it, 0.3500 is not
    assert AT.pick(table)[0] == [10, 2, 9, 1]


def test_pick_candidates_cover_every_window():
    plans = AT.candidates(0, 1, 50, True)
    assert {p[2] for p in plans} == set(AT.RB_CHOICES[(0, 1)])
    assert all(p[3] == 1 for p in plans)
    assert max(p[0] for p in plans) == 50
