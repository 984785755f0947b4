"""Pins of the physical beyond-dipole operator (input generator workloads/beyond.py; no GPU).

* Wigner 3j symbols: closed-form values and the orthogonality sum.
* H^theta_l (eq. Htheta) against a brute-force angular quadrature of
  4 pi Y_l0(z) <X_{-k1, mu1}| sigma_x Y_l0 |X_{k2, mu2}> with spinor harmonics built from scipy's
  spherical harmonics and Racah-formula Clebsch-Gordan coefficients (independent of the Gaunt /
  closed-form path of the generator); a swapped spin flip (sigma_z in place of sigma_x) fails.
* Selection rules of Sec. 2.4: every nonzero entry has mu' = mu +- 1 and an l inside the printed
  bounds. Reading: the printed bounds are the triangle rule of the orbital pair (l of kappa', l of
  -kappa), i.e. of H^theta_l with the two kappa arguments in the order opposite to eq. Htheta
  (with eq. Htheta's order, (kappa', kappa) = (-1, -2) couples through l = 0, which the printed
  bounds in that order would exclude).
* The factorisation of eq. bdpA: the six time functions times the Bessel radial functions and the
  Legendre angular factors reproduce the travelling sin^2 pulse at random points inside its window;
  a sign flip of the odd-l (cosine) part fails.
* The assembled coupling is Hermitian at random field values.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, roots_legendre
from scipy.special import sph_harm_y

from oracle.assemble import Assembled
from workloads import beyond as B
from workloads import dkb


def _racah_cg(j1, m1, j2, m2, J, M):
    if abs(m1 + m2 - M) > 1e-12:
        return 0.0
    f = math.factorial

    def fi(x):
        return f(int(round(x)))
    for x in (J + j1 - j2, J - j1 + j2, j1 + j2 - J, J + M, J - M, j1 - m1, j1 + m1, j2 - m2, j2 + m2):
        if x < -1e-9:
            return 0.0
    pre = math.sqrt((2 * J + 1) * fi(J + j1 - j2) * fi(J - j1 + j2) * fi(j1 + j2 - J) / fi(j1 + j2 + J + 1))
    pre *= math.sqrt(fi(J + M) * fi(J - M) * fi(j1 - m1) * fi(j1 + m1) * fi(j2 - m2) * fi(j2 + m2))
    s = 0.0
    for k in range(0, 60):
        args = [k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k]
        if any(a < -1e-9 for a in args):
            continue
        s += (-1) ** k / np.prod([fi(a) for a in args])
    return pre * s


def test_wigner_3j_values_and_orthogonality():
    assert abs(B.wigner_3j(1, 1, 0, 0, 0, 0) + 1 / math.sqrt(3)) < 1e-15
    assert abs(B.wigner_3j(2, 2, 2, 0, 0, 0) + math.sqrt(2.0 / 35.0)) < 1e-15
    assert abs(B.wigner_3j(1, 1, 2, 1, -1, 0) - math.sqrt(1.0 / 30.0)) < 1e-15
    j1, j2 = 2, 3
    for j3 in range(1, 6):
        for j3b in range(1, 6):
            for m3 in range(-min(j3, j3b), min(j3, j3b) + 1):
                tot = sum(B.wigner_3j(j1, j2, j3, m1, m2, m3) * B.wigner_3j(j1, j2, j3b, m1, m2, m3)
                          for m1 in range(-j1, j1 + 1) for m2 in range(-j2, j2 + 1))
                ref = (1.0 / (2 * j3 + 1)) if (j3 == j3b and abs(j1 - j2) <= j3 <= j1 + j2) else 0.0
                assert abs(tot - ref) < 1e-13


def _spinor(kappa, mu2, th, ph):
    """X_{kappa, mu} on the grid: (up, down) components from Racah CGs and scipy's Y_lm."""
    l = kappa if kappa > 0 else -kappa - 1
    j = abs(kappa) - 0.5
    mu = mu2 / 2.0
    up = _racah_cg(l, mu - 0.5, 0.5, 0.5, j, mu)
    dn = _racah_cg(l, mu + 0.5, 0.5, -0.5, j, mu)
    yu = sph_harm_y(l, int(round(mu - 0.5)), th, ph) if abs(mu - 0.5) <= l else 0 * th
    yd = sph_harm_y(l, int(round(mu + 0.5)), th, ph) if abs(mu + 0.5) <= l else 0 * th
    return up * yu, dn * yd


def _quadrature_htheta(l, k1, m1, k2, m2, flip="x"):
    x, wx = roots_legendre(24)
    th = np.arccos(x)
    nph = 32
    ph = 2 * np.pi * np.arange(nph) / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(wx, np.full(nph, 2 * np.pi / nph))
    a_up, a_dn = _spinor(-k1, m1, TH, PH)
    b_up, b_dn = _spinor(k2, m2, TH, PH)
    y = sph_harm_y(l, 0, TH, PH).real
    if flip == "x":
        integrand = np.conj(a_up) * y * b_dn + np.conj(a_dn) * y * b_up
    else:
        integrand = np.conj(a_up) * y * b_up - np.conj(a_dn) * y * b_dn
    val = np.sum(W * integrand)
    return (4 * np.pi * math.sqrt((2 * l + 1) / (4 * np.pi)) * val).real


def test_h_theta_matches_quadrature():
    rng = np.random.default_rng(3)
    kappas = [-1, 1, -2, 2, -3, 3]
    checked = nonzero = 0
    for _ in range(120):
        l = int(rng.integers(0, 4))
        k1, k2 = int(rng.choice(kappas)), int(rng.choice(kappas))
        m2 = int(rng.choice([m for m in range(-2 * abs(k2) + 1, 2 * abs(k2), 2)]))
        m1 = m2 + int(rng.choice([-2, 2]))
        if abs(m1) >= 2 * abs(k1):
            continue
        ref = _quadrature_htheta(l, k1, m1, k2, m2)
        got = B.h_theta(l, k1, m1, k2, m2)
        assert abs(got - ref) < 1e-12, (l, k1, m1, k2, m2, got, ref)
        checked += 1
        nonzero += abs(ref) > 1e-8
    assert checked > 60 and nonzero > 15
    # planted mistake: a sigma_z (no spin flip) angular factor differs wherever H^theta is nonzero
    planted = 0
    for l in range(0, 3):
        for k1 in kappas:
            for k2 in kappas:
                for m2 in range(-2 * abs(k2) + 1, 2 * abs(k2), 2):
                    m1 = m2 + 2
                    if abs(m1) >= 2 * abs(k1) or abs(B.h_theta(l, k1, m1, k2, m2)) < 1e-3 or planted >= 6:
                        continue
                    assert abs(_quadrature_htheta(l, k1, m1, k2, m2, flip="z") - B.h_theta(l, k1, m1, k2, m2)) > 1e-3
                    planted += 1
    assert planted == 6


def _paper_l_bounds(kp, k):
    """Bounds on l printed with the selection rules (row kappa', column kappa of H^theta_l)."""
    sg = lambda x: 1 if x > 0 else -1
    lo = abs(abs(-k) - abs(kp) + (sg(-k) - sg(kp)) / 2)
    hi = abs(-k) + abs(kp) + (sg(-k) + sg(kp)) / 2 - 1
    return lo, hi


def test_selection_rules():
    chans = B.channels(5, 5)
    for l in range(0, 5):
        A = B.angular_matrix_2(l, chans).tocoo()   # A[j'][j] = H^theta_l(kappa_j', kappa_j, mu_j', mu_j)
        assert A.nnz > 0
        for jp, j, v in zip(A.row, A.col, A.data):
            (kp, mp), (k, m) = chans[jp], chans[j]
            assert abs(mp - m) == 2
            lo, hi = _paper_l_bounds(k, kp)
            assert lo <= l <= hi, (l, kp, k)


def _pulse(E0, w, T, c, t, r, cth):
    tau = t - r * cth / c
    if not (0 < tau < T):
        return None
    return (E0 / w) * math.sin(math.pi * tau / T) ** 2 * math.sin(w * tau)


@pytest.mark.parametrize("sign", [1, -1])
def test_bdpA_factorisation_reproduces_the_pulse(sign):
    E0, w, cyc = 1.0, 1.0, 3
    T = cyc * 2 * math.pi / w
    c = dkb.C_LIGHT
    fs, meta = B.time_functions(w, T)
    rng = np.random.default_rng(9)
    err = 0.0
    n = 0
    for _ in range(400):
        t, r, cth = rng.uniform(0.5, T - 0.5), rng.uniform(0.0, 60.0), rng.uniform(-1.0, 1.0)
        ref = _pulse(E0, w, T, c, t, r, cth)
        if ref is None:
            continue
        val = 0.0
        for fi, (Om, wk, kind) in enumerate(meta):
            p = fs[fi]
            f = math.sin(p.omega * t + p.phase)
            for l in range(0, 14):
                g = B.radial_weight(l, Om, wk, kind, E0, w, np.array([r]), c)
                if g is None:
                    continue
                if kind == 1:
                    g = sign * g
                val += f * float(g[0]) * (2 * l + 1) * eval_legendre(l, cth)
        err = max(err, abs(val - ref))
        n += 1
    assert n > 300
    if sign == 1:
        assert err < 1e-12, err
    else:
        assert err > 1e-4  # planted mistake: the cosine (odd-l) part with the wrong sign


def test_assembled_coupling_is_hermitian():
    op, chans, basis, fs, T = B.hydrogen_beyond_dipole(nr=60, r_max=20.0, kappa_max=3, mu2_max=3, l_max=3)
    asm = Assembled(op)
    rng = np.random.default_rng(4)
    f = rng.standard_normal(op.n_fields)
    H = asm.hamiltonian(f)
    V = H - asm.H0
    d = V - V.conj().T
    assert abs(V).max() > 1e-3
    assert abs(d).max() <= 1e-12 * abs(V).max()
