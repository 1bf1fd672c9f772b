"""Host logic of the search driver (CPU): the progressive durations of Sec. II D."""
from paper_2510_20891_amd.search import progressive_durations


def test_progressive_durations_one_year():
    d = progressive_durations(192, 48)
    assert len(d) == 48                                  # 48 chunks, all distinct at 192 segments
    assert d[0] == round(0.1 * 192) and d[-1] == 192     # from 0.1 of the data to all of it
    steps = [b - a for a, b in zip(d, d[1:])]
    assert all(s > 0 for s in steps) and max(steps) - min(steps) <= 1    # near-equal growth


def test_progressive_durations_edges():
    assert progressive_durations(192, 1) == [192]
    d = progressive_durations(10, 48)                    # fewer segments than chunks: distinct, sorted
    assert d == sorted(set(d)) and d[0] == 1 and d[-1] == 10
    assert progressive_durations(631, 48)[0] == 63       # the paper's T_SFT = 5e4 s year (631 segments)
