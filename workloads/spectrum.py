"""Inputs of the photoelectron-spectrum path: the hydrogen DKB operator, the field-free eigenpairs of
every distinct kappa block inside an energy window (computed before the run, as the paper's
pre-computed input), an energy grid, and a driven state to analyse.

The eigen-decomposition is input preparation (LAPACK via scipy, dense generalised symmetric
problem per kappa); the spectrum itself (projection, density, interpolation, sum over channels)
is the library's. The oracle diagonalises the same blocks on its own.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla

from . import dkb
from .desc import Pulse, Workload


@dataclasses.dataclass
class SpectrumInputs:
    blk_of: np.ndarray    # [nang] eigen-block of every channel
    n_lev: np.ndarray     # [n_blk]
    levels: np.ndarray    # concatenated levels inside the window, ascending per block
    edges: np.ndarray     # [n_blk][2] nearest levels below / above the window
    vecs: np.ndarray      # [total levels][2 nr] real eigenvectors, v^T S v = 1
    grid: np.ndarray      # [n_grid]
    e_lo: float
    e_hi: float


def eigen_inputs(op, e_lo: float, e_hi: float, grid: np.ndarray) -> SpectrumInputs:
    kap_vals = sorted(set(float(k) for k in op.kappa))
    blk_index = {k: b for b, k in enumerate(kap_vals)}
    blk_of = np.array([blk_index[float(k)] for k in op.kappa], dtype=np.int32)
    n_lev, levels, edges, vecs = [], [], [], []
    for k in kap_vals:
        H = dkb.dense_block(op.h_poly, k, op.nr, op.hb)
        S = dkb.dense_block(op.s_poly, k, op.nr, op.hb)
        E, V = sla.eigh(H, S)
        sel = np.nonzero((E > e_lo) & (E < e_hi))[0]
        assert len(sel) > 0 and sel[0] > 0 and sel[-1] + 1 < len(E), "window must lie inside the spectrum"
        n_lev.append(len(sel))
        levels.append(E[sel])
        edges.append([E[sel[0] - 1], E[sel[-1] + 1]])
        vecs.append(V[:, sel].T)
    return SpectrumInputs(blk_of, np.array(n_lev, dtype=np.int32), np.concatenate(levels),
                          np.array(edges, dtype=np.float64), np.ascontiguousarray(np.concatenate(vecs, 0)),
                          np.asarray(grid, dtype=np.float64), e_lo, e_hi)


def hydrogen_case(nr: int = 600, r_max: float = 60.0, lmax: int = 10, e_lo: float = 0.02, e_hi: float = 3.0,
                  n_grid: int = 300, E0: float = 1.0, omega: float = 1.0, cycles: int = 4, dt: float = 2e-3):
    """Hydrogen DKB operator on [0, r_max] (the paper's physical-validation box, Sec. 4.x), channels
    l <= lmax at mu = 1/2, the ground state and a sin^2 pulse (A = (E0/w) sin^2 sin) of `cycles`
    cycles whose steps the caller runs to ionise it; eigen-inputs on a grid inside (e_lo, e_hi).
    Returns (workload, SpectrumInputs)."""
    w = dkb.config2(nr=nr, r_max=r_max, lmax=lmax, E0=E0, omega=omega, cycles=cycles, dt=dt)
    T = cycles * 2 * math.pi / omega
    n_steps = int(round(T / dt))
    w = dataclasses.replace(w, n_steps=np.array([n_steps], dtype=np.int32),
                            pulses=[[Pulse(amp=E0 / omega, T=T, omega=omega, phase=0.0, envelope=True)]])
    grid = np.linspace(e_lo + 0.03, e_hi - 0.03, n_grid)
    return w, eigen_inputs(w.op, e_lo, e_hi, grid)
