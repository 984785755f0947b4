"""Crank-Nicolson time step (oracle).

Paper eq. solPsi with the midpoint rule of Sec. 2.4 (the Hamiltonian of the step
(t_n, t_n + dt) is taken at t_n + dt/2, which gives the O(dt^2) propagator the text
derives):

    (S + i dt/2 H(t_mid)) psi_{n+1} = (S - i dt/2 H(t_mid)) psi_n

solved by BiCGSTAB (``bicgstab``) or, for checks, by a dense / sparse direct solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .assemble import Assembled
from .bicgstab import bicgstab
from .fields import field_values, midpoint_time


def step_matrices(asm: Assembled, fvals, dt: float):
    """(A, B) = (S + i dt/2 H, S - i dt/2 H)."""
    H = asm.hamiltonian(fvals)
    A = (asm.S + (0.5j * dt) * H).tocsr()
    B = (asm.S - (0.5j * dt) * H).tocsr()
    return A, B


class BlockPreconditioner:
    """LU factors of the block-diagonal M = S + i dt/2 H0 (paper eq. matrixM), factored once per dt."""

    def __init__(self, asm: Assembled, dt: float):
        self.dt = dt
        M = (asm.S + (0.5j * dt) * asm.H0).tocsc()
        self.lu = spla.splu(M)

    def __call__(self, z):
        return self.lu.solve(z)


def cn_step(asm: Assembled, pulses_row, t_n: float, dt: float, psi: np.ndarray, guess: str | np.ndarray = "prev",
            tol: float = 1e-12, max_iter: int = 2000, solver: str = "bicgstab", precond=None):
    """One step psi_n -> psi_{n+1} of one instance. psi: complex [nang][2][nr] (or flat).

    guess: "prev" (x0 = psi_n), "zero", or an explicit array. solver: "bicgstab", "dense"
    (LAPACK LU) or "splu" (sparse LU). precond: None or a ``BlockPreconditioner`` for this dt.
    Returns (psi_{n+1}, stats or None).
    """
    shape = psi.shape
    f = field_values(pulses_row, midpoint_time(t_n, dt))
    A, B = step_matrices(asm, f, dt)
    b = B @ psi.ravel()
    if solver == "dense":
        return np.linalg.solve(A.toarray(), b).reshape(shape), None
    if solver == "splu":
        return spla.splu(A.tocsc()).solve(b).reshape(shape), None
    if isinstance(guess, str):
        x0 = psi.ravel().copy() if guess == "prev" else np.zeros_like(b)
    else:
        x0 = np.asarray(guess).ravel()
    x, st = bicgstab(A, b, x0, tol, max_iter, precond)
    return x.reshape(shape), st


def propagate(asm: Assembled, pulses_row, t0: float, dt: float, psi0: np.ndarray, n_steps: int, **kw):
    """n_steps consecutive steps; returns (final state, list of per-step stats)."""
    psi = psi0.copy()
    stats = []
    for n in range(n_steps):
        psi, st = cn_step(asm, pulses_row, t0 + n * dt, dt, psi, **kw)
        stats.append(st)
    return psi, stats
