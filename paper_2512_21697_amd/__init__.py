"""MI355X (gfx950) Crank-Nicolson / BiCGSTAB time step for the time-dependent Dirac equation.

The compute path is the HIP library libtdde.so (C ABI in include/tdde.h); ``_lib`` is its ctypes
binding. PyTorch only provides device memory and streams.
"""
from ._lib import (GUESS_GIVEN, GUESS_PREV, GUESS_ZERO, PREC_FP64, PREC_MIXED, STATS_DTYPE, TDDE_BREAKDOWN,
                   TDDE_NONFINITE, TDDE_NOT_CONVERGED, TDDE_OK, Net, Solver, TddeError, load, solve_opts)

__all__ = ["Solver", "Net", "TddeError", "load", "solve_opts", "GUESS_ZERO", "GUESS_PREV", "GUESS_GIVEN", "PREC_FP64",
           "PREC_MIXED", "STATS_DTYPE", "TDDE_OK", "TDDE_NOT_CONVERGED", "TDDE_BREAKDOWN", "TDDE_NONFINITE"]
