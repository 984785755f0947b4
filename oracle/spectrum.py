"""Photoelectron energy spectrum and the spectral error (oracle; test infrastructure).

Eq. dPdE: dP/dE = sum over channels (kappa, mu) of |<psi_{kappa,mu,E}|Psi>|^2, with psi_{kappa,mu,E}
the field-free eigenstates of the channel's radial block, found by diagonalisation (Sec. 2.3: the
generalised problem H0_kappa v = E S_kappa v; the angular part is the channel's spinor, so the
overlap with Psi reduces to the channel's radial coefficients). In a finite box the positive-energy
states are discrete; a box-normalised eigenvector v_n (v_n^T S v_n = 1) stands for the
energy-normalised state times sqrt(dE_n), dE_n the local level spacing (reading), so at E = E_n

    dP/dE (E_n) = |v_n^T S Psi_j|^2 / dE_n,   dE_n = (E_{n+1} - E_{n-1}) / 2.

Each channel's values, on its own levels inside the energy window, are interpolated linearly onto a
common energy grid (zero outside the channel's first and last level in the window) and summed over
channels. The error of a spectrum P_n against a reference P_m (Sec. 4.x, convergence) is
Err = integral over [E1, E2] of |P_n - P_m|^2 dE, here by the trapezoidal rule on the grid.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .assemble import kappa_poly_block


def block_matrices(op, kappa: float):
    """Dense (H0, S) of one channel's radial block ([2 nr] x [2 nr], rows s * nr + i)."""
    H = kappa_poly_block(op.h_poly, kappa, op.nr, op.hb).toarray()
    if op.s_poly.shape[0]:
        S = kappa_poly_block(op.s_poly, kappa, op.nr, op.hb).toarray()
    else:
        S = np.eye(2 * op.nr)
    return H, S


def eigenpairs(H: np.ndarray, S: np.ndarray):
    """Generalised symmetric eigenproblem H v = E S v: (E ascending, V with V^T S V = I)."""
    E, V = sla.eigh(H, S)
    return E, V


def level_spacing(E: np.ndarray) -> np.ndarray:
    """dE_n = (E_{n+1} - E_{n-1}) / 2, one-sided at the first and last level."""
    d = np.empty_like(E)
    d[1:-1] = 0.5 * (E[2:] - E[:-2])
    d[0] = E[1] - E[0]
    d[-1] = E[-1] - E[-2]
    return d


def channel_density(E, V, S, psi_j, e_lo, e_hi):
    """(levels in (e_lo, e_hi), dP/dE at those levels) of one channel; psi_j: [2 nr] radial coefficients."""
    dE = level_spacing(E)
    sel = (E > e_lo) & (E < e_hi)
    c = V[:, sel].T @ (S @ psi_j)
    return E[sel], np.abs(c) ** 2 / dE[sel]


def on_grid(levels, dens, grid):
    """Linear interpolation of one channel's density onto the grid; zero outside its levels."""
    if len(levels) == 0:
        return np.zeros_like(grid)
    return np.interp(grid, levels, dens, left=0.0, right=0.0)


def spectrum(op, psi, grid, e_lo, e_hi):
    """dP/dE on the grid for a state psi [nang][2][nr] (sum over channels; real kappa-polynomial
    operators only: the channel blocks must be real symmetric)."""
    assert op.h_chan is None, "per-channel complex bands: the eigenvectors would be complex"
    psi = np.asarray(psi).reshape(op.nang, 2 * op.nr)
    out = np.zeros(len(grid))
    cache = {}
    for j in range(op.nang):
        kap = float(op.kappa[j])
        if kap not in cache:
            H, S = block_matrices(op, kap)
            E, V = eigenpairs(H, S)
            cache[kap] = (E, V, S)
        E, V, S = cache[kap]
        lv, dn = channel_density(E, V, S, psi[j], e_lo, e_hi)
        out += on_grid(lv, dn, grid)
    return out


def spectral_error(p1, p2, grid):
    """Err = integral of |p1 - p2|^2 dE over the grid (trapezoidal rule)."""
    d = np.abs(np.asarray(p1) - np.asarray(p2)) ** 2
    return float(np.sum(0.5 * (d[1:] + d[:-1]) * np.diff(grid)))
