"""Launch-shape autotuner for the persistent solver kernel.

The persistent kernel runs on a grid of co-resident work-groups; how many share one compute unit is
a trade between latency hiding (more waves in flight per CU for the banded applies and the
preconditioner's substitution chains) and the cost of the grid-wide barriers of every BiCGSTAB
iteration (every work-group arrives at each one). The best point depends on the operator size and
the batch, so it is measured, not fixed: ``tune_launch`` times a caller-supplied piece of work
under every candidate shape and leaves the solver on the fastest one.

Host code here only selects and times; the work itself runs in the library.
"""
from __future__ import annotations

import time
from typing import Callable, Dict, Iterable, Tuple

from ._lib import TddeError


def tune_launch(solver, run: Callable[[], None], candidates: Iterable[int] = (1, 2, 3, 4), reps: int = 3,
                sync: Callable[[], None] = None, prefer: int = None,
                margin: float = 0.02) -> Tuple[int, Dict[int, float]]:
    """Time ``run()`` under each launch shape (work-groups per CU) and keep the fastest.

    ``run`` launches a fixed piece of work on ``solver`` (for example one persistent chunk of steps
    on a scratch copy of the state); it is called once untimed per shape, then ``reps`` times under
    the timer, and the median is kept. ``sync`` waits for the device (default: torch's
    ``cuda.synchronize``). Shapes the library rejects (fewer work-groups than instances) are
    skipped. ``prefer`` (if given and timed) is kept unless another shape is faster by more than
    the fraction ``margin``, so that timing noise between near-equal shapes does not flip the
    choice from run to run. Returns (chosen shape, {shape: median seconds}); the solver is left
    on the chosen shape.
    """
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    times: Dict[int, float] = {}
    for k in candidates:
        try:
            solver.set_launch(k)
        except TddeError:
            continue
        run()
        sync()
        samples = []
        for _ in range(max(1, reps)):
            t0 = time.perf_counter()
            run()
            sync()
            samples.append(time.perf_counter() - t0)
        samples.sort()
        times[k] = samples[len(samples) // 2]
    if not times:
        raise TddeError(-1, "no launch shape accepted")
    best = min(times, key=times.get)
    if prefer in times and times[best] >= (1.0 - margin) * times[prefer]:
        best = prefer
    solver.set_launch(best)
    return best, times
