"""Host logic of the launch-shape autotuner, on a stand-in solver (no GPU)."""
import time

import pytest

from paper_2512_21697_amd._lib import TddeError
from paper_2512_21697_amd.autotune import tune_launch


class _FakeSolver:
    """Accepts shapes 1..3 (4 is rejected as too small a grid would be); runs take a time set by
    the current shape."""

    def __init__(self, cost):
        self.cost, self.shape, self.calls = cost, 0, []

    def set_launch(self, k):
        if k not in self.cost:
            raise TddeError(-1, "rejected")
        self.shape = k

    def run(self):
        self.calls.append(self.shape)
        time.sleep(self.cost[self.shape])


def test_picks_fastest_and_skips_rejected():
    s = _FakeSolver({1: 0.012, 2: 0.002, 3: 0.008})
    best, times = tune_launch(s, s.run, candidates=(1, 2, 3, 4), reps=3, sync=lambda: None)
    assert best == 2 and s.shape == 2
    assert set(times) == {1, 2, 3}
    assert times[2] < times[3] < times[1]
    # one untimed run and three timed runs per accepted shape
    assert [s.calls.count(k) for k in (1, 2, 3)] == [4, 4, 4]


def test_no_accepted_shape_raises():
    s = _FakeSolver({})
    with pytest.raises(TddeError):
        tune_launch(s, s.run, candidates=(1, 2), sync=lambda: None)


def test_preferred_shape_kept_within_margin():
    s = _FakeSolver({1: 0.010, 2: 0.0099, 4: 0.010})
    best, _ = tune_launch(s, s.run, candidates=(1, 2, 4), reps=1, sync=lambda: None, prefer=4, margin=0.2)
    assert best == 4 and s.shape == 4
    s = _FakeSolver({1: 0.010, 2: 0.002, 4: 0.010})
    best, _ = tune_launch(s, s.run, candidates=(1, 2, 4), reps=1, sync=lambda: None, prefer=4, margin=0.2)
    assert best == 2 and s.shape == 2
