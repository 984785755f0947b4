"""Textbook complex BiCGSTAB, optionally right-preconditioned (oracle).

The iterative solver of paper Sec. 2.4 / Sec. 3.3, written out as in van der Vorst,
SIAM J. Sci. Stat. Comput. 13 (1992) 631, with inner product <a, b> = sum conj(a) b.
With a preconditioner K (paper eq. matrixM: K = M = S + i dt/2 H0, applied through its
LU factors) the search directions are p_hat = K^-1 p and s_hat = K^-1 s, A acts on
those, and x is updated with them; r stays the residual of the original system.
Stopping rule: ||r|| <= tol ||b|| on the recursive residual (also tested on s after
the half step), then the true residual b - A x is checked once; if it fails, the
iteration restarts from the current x. A vanishing rho, <r^, v> or omega restarts with
r^ = r (van der Vorst leaves the shadow residual r^ free as long as <r^, r0> != 0; a
restart is the standard remedy when one of the three scalars becomes zero).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class SolveStats:
    iters: int = 0  # full iterations (a half step counts as one)
    matvecs: int = 0
    restarts: int = 0
    rel_res: float = 0.0  # recursive residual at exit
    true_rel_res: float = 0.0
    converged: bool = False


def _dot(a, b):
    return np.vdot(a, b)


def bicgstab(A, b: np.ndarray, x0: np.ndarray | None, tol: float = 1e-12, max_iter: int = 1000, precond=None,
             rhat0: np.ndarray | None = None, max_restarts: int = 20):
    """Solve A x = b. A is anything with ``@`` (scipy sparse or dense); precond is None or a
    callable z -> K^-1 z. rhat0: shadow residual of the first cycle (default r0; later cycles
    after a restart always take r^ = r). More than max_restarts restarts end the solve
    unconverged (a Krylov space that breaks down again after every restart makes no progress).
    Returns (x, SolveStats)."""
    apply_k = (lambda z: z) if precond is None else precond
    st = SolveStats()
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        st.converged = True
        return np.zeros_like(b), st
    target = tol * bnorm
    r = b - A @ x
    st.matvecs += 1
    if np.linalg.norm(r) <= target:
        st.converged = True
        st.rel_res = st.true_rel_res = np.linalg.norm(r) / bnorm
        return x, st
    first_cycle = True
    while True:
        rhat = r.copy() if (rhat0 is None or not first_cycle) else np.asarray(rhat0, dtype=np.complex128).copy()
        first_cycle = False
        rho_old = alpha = omega = 1.0 + 0.0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        done = False
        while st.iters < max_iter:
            rho = _dot(rhat, r)
            if abs(rho) < 1e-300 * (1.0 + np.linalg.norm(rhat) * np.linalg.norm(r)):
                st.restarts += 1
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = apply_k(p)
            v = A @ ph
            st.matvecs += 1
            rv = _dot(rhat, v)
            if rv == 0:
                st.restarts += 1
                break
            alpha = rho / rv
            s = r - alpha * v
            st.iters += 1
            if np.linalg.norm(s) <= target:
                x = x + alpha * ph
                st.rel_res = np.linalg.norm(s) / bnorm
                done = True
                break
            sh = apply_k(s)
            t = A @ sh
            st.matvecs += 1
            tt = _dot(t, t).real
            omega = _dot(t, s) / tt if tt > 0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rn = np.linalg.norm(r)
            st.rel_res = rn / bnorm
            if rn <= target:
                done = True
                break
            if omega == 0:
                st.restarts += 1
                break
            rho_old = rho
        if st.iters >= max_iter and not done:
            break
        # true-residual check (a failed check restarts from the current iterate)
        r = b - A @ x
        st.matvecs += 1
        st.true_rel_res = np.linalg.norm(r) / bnorm
        if done and st.true_rel_res <= tol:
            st.converged = True
            break
        if st.iters >= max_iter:
            break
        if done:
            st.restarts += 1
        if st.restarts > max_restarts:
            break
    if not st.converged:
        r = b - A @ x
        st.true_rel_res = np.linalg.norm(r) / bnorm
    return x, st
