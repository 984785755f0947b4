"""Pins of the oracle's photoelectron spectrum (eq. dPdE) and its error integral (no GPU).

* Completeness: summed over every eigenstate of a channel block, the probabilities |v_n^T S psi|^2
  add up to the S-norm psi^H S psi (hydrogen DKB block, S != I): a projection without S or with a
  wrong normalisation fails.
* An eigenvector as the state projects onto that eigenvector alone.
* A model block with closed-form eigenpairs (finite-difference -1/2 d^2/dx^2 in a box):
  E_n = (1 - cos(n pi / (N + 1))) / h^2, v_n = sqrt(2 / (N + 1)) sin(n j pi / (N + 1)). A state built
  as sum_n g(E_n) sqrt(dE_n) v_n has the density g(E)^2, so the oracle's spectrum of it must return
  g^2 on the grid (g^2 linear in E: the interpolation is exact); a missing 1/dE or a one-sided spacing
  fails.
* The error integral: zero for equal spectra, a^2 (E2 - E1) for a constant difference a, quadratic
  scaling, and the trapezoidal value of a linear difference.
"""
import math

import numpy as np
import pytest

from oracle import spectrum as S
from workloads import dkb


def _hydrogen_block(nr=60, kappa=-1.0):
    op, _, _ = dkb.hydrogen_operator(nr=nr, r_max=30.0, lmax=1)
    return S.block_matrices(op, kappa)


@pytest.mark.parametrize("kappa", [-1.0, 2.0])
def test_completeness_is_the_s_norm(kappa):
    H, Sm = _hydrogen_block(kappa=kappa)
    assert np.max(np.abs(Sm - np.eye(len(Sm)))) > 1e-3  # S is not the identity
    E, V = S.eigenpairs(H, Sm)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal(len(H)) + 1j * rng.standard_normal(len(H))
    c = V.T @ (Sm @ psi)
    norm = np.vdot(psi, Sm @ psi).real
    assert abs(np.sum(np.abs(c) ** 2) - norm) <= 1e-10 * norm
    # the same sum through the density: |c|^2 / dE times dE, over a window holding every level
    lv, dn = S.channel_density(E, V, Sm, psi, E[0] - 1.0, E[-1] + 1.0)
    assert abs(np.sum(dn * S.level_spacing(E)) - norm) <= 1e-10 * norm
    # planted mistake: the projection without the overlap does not conserve the norm
    assert abs(np.sum(np.abs(V.T @ psi) ** 2) - norm) > 1e-3 * norm


def test_eigenvector_projects_onto_itself():
    H, Sm = _hydrogen_block()
    E, V = S.eigenpairs(H, Sm)
    k = int(np.searchsorted(E, 0.5))
    c = V.T @ (Sm @ V[:, k])
    ref = np.zeros(len(E))
    ref[k] = 1.0
    assert np.max(np.abs(c - ref)) < 1e-10


def _box(N=400, L=40.0):
    h = L / (N + 1)
    H = np.diag(np.full(N, 1.0 / h ** 2)) + np.diag(np.full(N - 1, -0.5 / h ** 2), 1) + \
        np.diag(np.full(N - 1, -0.5 / h ** 2), -1)
    n = np.arange(1, N + 1)
    E = (1.0 - np.cos(n * math.pi / (N + 1))) / h ** 2
    j = np.arange(1, N + 1)
    V = math.sqrt(2.0 / (N + 1)) * np.sin(np.outer(j, n) * math.pi / (N + 1))
    return H, E, V


def test_box_eigenpairs_closed_form():
    H, E, V = _box()
    Eo, Vo = S.eigenpairs(H, np.eye(len(H)))
    assert np.max(np.abs(Eo - E)) < 1e-9 * E.max()
    # eigenvectors up to sign
    sgn = np.sign(np.sum(Vo * V, axis=0))
    assert np.max(np.abs(Vo * sgn - V)) < 1e-8


def test_box_density_normalisation():
    H, E, V = _box()
    dE = np.empty_like(E)
    dE[1:-1] = 0.5 * (E[2:] - E[:-2])
    dE[0], dE[-1] = E[1] - E[0], E[-1] - E[-2]
    assert np.allclose(S.level_spacing(E), dE, rtol=0, atol=1e-12)
    g2 = lambda e: 0.3 + 0.1 * e  # a density linear in E
    psi = V @ (np.sqrt(g2(E) * dE) * np.exp(1j * 0.7 * np.arange(len(E))))
    e_lo, e_hi = 0.5, 3.0
    grid = np.linspace(0.6, 2.9, 57)
    lv, dn = S.channel_density(E, V, np.eye(len(E)), psi, e_lo, e_hi)
    assert np.max(np.abs(dn - g2(lv))) < 1e-10
    on = S.on_grid(lv, dn, grid)
    assert np.max(np.abs(on - g2(grid))) < 1e-10
    # planted mistakes: no division by the spacing, or a one-sided spacing
    assert np.max(np.abs(np.abs(V.T @ psi)[(E > e_lo) & (E < e_hi)] ** 2 - g2(lv))) > 1e-3
    one_sided = np.abs(V.T @ psi) ** 2 / np.append(np.diff(E), E[-1] - E[-2])
    assert np.max(np.abs(one_sided[(E > e_lo) & (E < e_hi)] - g2(lv))) > 1e-5


def test_spectral_error_integral():
    grid = np.linspace(0.2, 3.4, 101)
    rng = np.random.default_rng(2)
    p = rng.uniform(0, 1, grid.size)
    assert S.spectral_error(p, p, grid) == 0.0
    a = 0.37
    assert abs(S.spectral_error(p + a, p, grid) - a * a * (grid[-1] - grid[0])) < 1e-12
    q = rng.uniform(0, 1, grid.size)
    assert abs(S.spectral_error(3 * p, 3 * q, grid) - 9 * S.spectral_error(p, q, grid)) < 1e-12
    # linear difference alpha * E: trapezoid of alpha^2 E^2 on a uniform grid
    al = 0.8
    h = grid[1] - grid[0]
    exact = al * al * (grid[-1] ** 3 - grid[0] ** 3) / 3.0
    trap = exact + al * al * h * h * (grid[-1] - grid[0]) / 6.0  # trapezoid error of E^2: + h^2 (b - a) / 6
    assert abs(S.spectral_error(p + al * grid, p, grid) - trap) < 1e-10
