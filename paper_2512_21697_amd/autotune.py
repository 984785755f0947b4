"""Autotuner for the solver's launch knobs.

Three knobs are measured rather than fixed, because the best point depends on the operator size and the
batch:
  * the solver form: one persistent cooperative launch per chunk of steps, or one kernel per window of
    the iteration (each at its own occupancy; pays a launch and a host read per iteration);
  * the persistent grid's shape (work-groups per CU): latency hiding (more waves in flight for the
    banded applies and the preconditioner's substitution chains) against the cost of the grid-wide
    barriers every work-group takes part in. Kernel variants cap the shape by their occupancy, so
    several requested shapes can launch the same grid; those are timed once.
  * the preconditioner's segment length (rows per thread of the segmented triangular solves):
    longer segments mean fewer boundary matrices but longer sequential chains.
``tune_launch``, ``tune_form`` and ``tune_segment`` time a caller-supplied piece of work (one persistent chunk of
steps on a scratch copy of the state) under every candidate and leave the solver on the fastest.

Host code here only selects and times; the work itself runs in the library.
"""
from __future__ import annotations

import time
from typing import Callable, Dict, Iterable, Tuple

from ._lib import TddeError


def _median_time(run, sync, reps):
    run()
    sync()
    samples = []
    for _ in range(max(1, reps)):
        t0 = time.perf_counter()
        run()
        sync()
        samples.append(time.perf_counter() - t0)
    samples.sort()
    return samples[len(samples) // 2]


def _pick(times, prefer, margin):
    best = min(times, key=times.get)
    if prefer in times and times[best] >= (1.0 - margin) * times[prefer]:
        best = prefer
    return best


def tune_launch(solver, run: Callable[[], None], candidates: Iterable[int] = (1, 2, 3, 4), reps: int = 3,
                sync: Callable[[], None] = None, prefer: int = None,
                margin: float = 0.02) -> Tuple[int, Dict[int, float], Dict[int, int]]:
    """Time ``run()`` under each launch shape (work-groups per CU) and keep the fastest.

    ``run`` launches a fixed piece of work on ``solver``; it is called once untimed per shape, then
    ``reps`` times under the timer, and the median is kept. ``sync`` waits for the device (default:
    torch's ``cuda.synchronize``). Shapes the library rejects are skipped; a shape whose launches use
    the same grid (work-groups actually launched, read after the first run) as a shape already timed
    shares that timing instead of being timed again. ``prefer`` (if given and timed) is kept unless
    another shape is faster by more than the fraction ``margin``, so that timing noise between
    near-equal shapes does not flip the choice. Returns (chosen shape, {shape: median seconds},
    {shape: grid}); the solver is left on the chosen shape."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    times: Dict[int, float] = {}
    grids: Dict[int, int] = {}
    by_grid: Dict[int, float] = {}
    for k in candidates:
        try:
            solver.set_launch(k)
        except TddeError:
            continue
        run()
        sync()
        grid = solver.launch_info()[0]
        grids[k] = grid
        if grid not in by_grid:
            by_grid[grid] = _median_time(run, sync, reps)
        times[k] = by_grid[grid]
    if not times:
        raise TddeError(-1, "no launch shape accepted")
    # among shapes with the same grid the smallest request stands for it
    distinct = {}
    for k in sorted(times):
        distinct.setdefault(grids[k], k)
    cand = {k: times[k] for k in distinct.values()}
    best = _pick(cand, prefer if prefer in cand else None, margin)
    if prefer in times and grids[prefer] == grids[best]:
        best = prefer
    solver.set_launch(best)
    return best, times, grids


def tune_segment(solver, dt: float, run: Callable[[], None], candidates: Iterable[int] = (24, 32, 48, 64),
                 reps: int = 3, sync: Callable[[], None] = None, prefer: int = None,
                 margin: float = 0.02) -> Tuple[int, Dict[int, float]]:
    """Time ``run()`` with each least segment length of the preconditioner (refactoring at ``dt`` for
    each) and keep the fastest (``prefer`` kept within ``margin``, as in ``tune_launch``). Returns
    (chosen length, {length: median seconds}); the solver is left factored with the chosen length."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    times: Dict[int, float] = {}
    for m in candidates:
        try:
            solver.set_prec_segment(m)
            solver.set_dt(dt)
        except TddeError:
            continue
        times[m] = _median_time(run, sync, reps)
    if not times:
        raise TddeError(-1, "no segment length accepted")
    best = _pick(times, prefer, margin)
    solver.set_prec_segment(best)
    solver.set_dt(dt)
    return best, times


def tune_form(solver, run: Callable[[], None], reps: int = 3, sync: Callable[[], None] = None,
              prefer: str = None, margin: float = 0.02) -> Tuple[str, Dict[str, float]]:
    """Time ``run()`` in the persistent form (on the solver's current launch shape) and in the
    kernel-per-window form, and keep the faster (``prefer`` kept within ``margin``). Returns
    (chosen form, {form: median seconds}); the solver is left on the chosen form."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    times: Dict[str, float] = {}
    for form in ("persistent", "split"):
        try:
            solver.set_split(form == "split")
        except TddeError:
            continue
        times[form] = _median_time(run, sync, reps)
    if not times:
        raise TddeError(-1, "no solver form accepted")
    best = _pick(times, prefer, margin)
    solver.set_split(best == "split")
    return best, times
