"""Host logic of the autotuner (launch shape and preconditioner segment length), on a stand-in
solver (no GPU)."""
import time

import pytest

from paper_2512_21697_amd._lib import TddeError
from paper_2512_21697_amd.autotune import tune_launch, tune_segment


class _FakeSolver:
    """Accepts the shapes in ``cost``; a shape launches the grid ``grid[shape]`` (default 256 * shape);
    runs take the time set by the current shape / segment length."""

    def __init__(self, cost, grid=None, seg_cost=None):
        self.cost, self.shape, self.calls = cost, 0, []
        self.grid = grid or {k: 256 * k for k in cost}
        self.seg_cost, self.seg, self.dt = seg_cost or {}, None, None

    def set_launch(self, k):
        if k not in self.cost:
            raise TddeError(-1, "rejected")
        self.shape = k

    def launch_info(self):
        return self.grid[self.shape], self.grid[self.shape]

    def set_prec_segment(self, m):
        if m not in self.seg_cost:
            raise TddeError(-1, "rejected")
        self.seg = m

    def set_dt(self, dt):
        self.dt = dt

    def run(self):
        self.calls.append(self.shape)
        time.sleep(self.seg_cost[self.seg] if self.seg is not None else self.cost[self.shape])


def test_picks_fastest_and_skips_rejected():
    s = _FakeSolver({1: 0.012, 2: 0.002, 3: 0.008})
    best, times, grids = tune_launch(s, s.run, candidates=(1, 2, 3, 4), reps=3, sync=lambda: None)
    assert best == 2 and s.shape == 2
    assert set(times) == {1, 2, 3}
    assert times[2] < times[3] < times[1]
    assert grids == {1: 256, 2: 512, 3: 768}
    # two untimed runs (the grid read and the warm-up) and three timed runs per accepted shape
    assert [s.calls.count(k) for k in (1, 2, 3)] == [5, 5, 5]


def test_shapes_with_the_same_grid_are_timed_once():
    s = _FakeSolver({1: 0.012, 2: 0.002, 3: 0.002, 4: 0.002}, grid={1: 256, 2: 512, 3: 512, 4: 512})
    best, times, grids = tune_launch(s, s.run, candidates=(1, 2, 3, 4), reps=2, sync=lambda: None, prefer=4)
    assert times[2] == times[3] == times[4]
    assert [s.calls.count(k) for k in (1, 2, 3, 4)] == [4, 4, 1, 1]
    assert best == 4  # the preferred shape launches the winning grid


def test_no_accepted_shape_raises():
    s = _FakeSolver({})
    with pytest.raises(TddeError):
        tune_launch(s, s.run, candidates=(1, 2), sync=lambda: None)


def test_preferred_shape_kept_within_margin():
    s = _FakeSolver({1: 0.010, 2: 0.0099, 4: 0.010})
    best, _, _ = tune_launch(s, s.run, candidates=(1, 2, 4), reps=1, sync=lambda: None, prefer=4, margin=0.2)
    assert best == 4 and s.shape == 4
    s = _FakeSolver({1: 0.010, 2: 0.002, 4: 0.010})
    best, _, _ = tune_launch(s, s.run, candidates=(1, 2, 4), reps=1, sync=lambda: None, prefer=4, margin=0.2)
    assert best == 2 and s.shape == 2


def test_segment_length_tuning_refactors_and_keeps_fastest():
    s = _FakeSolver({4: 0.001}, seg_cost={24: 0.008, 32: 0.003, 48: 0.006})
    best, times = tune_segment(s, 1e-3, s.run, candidates=(16, 24, 32, 48), reps=2, sync=lambda: None, prefer=24)
    assert best == 32 and s.seg == 32 and s.dt == 1e-3
    assert set(times) == {24, 32, 48}


class _FormSolver:
    def __init__(self, cost):
        self.cost, self.split = cost, False

    def set_split(self, on):
        self.split = bool(on)

    def run(self):
        time.sleep(self.cost["split" if self.split else "persistent"])


def test_form_picks_faster_and_prefers_within_margin():
    from paper_2512_21697_amd.autotune import tune_form
    s = _FormSolver({"persistent": 0.010, "split": 0.004})
    best, times = tune_form(s, s.run, reps=2, sync=lambda: None)
    assert best == "split" and s.split and times["split"] < times["persistent"]
    s = _FormSolver({"persistent": 0.0100, "split": 0.0099})
    best, _ = tune_form(s, s.run, reps=2, sync=lambda: None, prefer="persistent", margin=0.2)
    assert best == "persistent" and not s.split
