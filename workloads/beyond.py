"""Physical beyond-dipole coupling of the hydrogen DKB operator: a linearly polarised sin^2 pulse
propagating along z with polarisation along x (eq. ndpPot), its factorisation into six time
functions and Bessel radial functions (eq. bdpA), the angular matrices H^theta_l of eq. Htheta
from spin-1/2 Clebsch-Gordan coefficients and Gaunt integrals (eq. HthetaExpand, eq. GauntCoef), and
the kappa-bilinear radial projections of eq. fullH. Input generation only (the time step is the
library's; the oracle assembles the same description into CSR on its own).

Time functions and radial functions (eq. bdpA). With tau = t - z/c and W = 2 pi / T,
  sin^2(pi tau / T) sin(w tau) = 1/2 sin(w tau) - 1/4 sin((w + W) tau) - 1/4 sin((w - W) tau),
  sin(O (t - z/c)) = sin(O t) cos(O z / c) - cos(O t) sin(O z / c),
and the plane-wave expansion (k along z)
  cos(q z) = sum_{l even} (-1)^{l/2} (2l+1) j_l(q r) P_l(cos theta),
  sin(q z) = sum_{l odd} (-1)^{(l-1)/2} (2l+1) j_l(q r) P_l(cos theta),
with (2l+1) P_l(cos theta) = 4 pi Y_l0(z^) Y_l0(r^). So
  A_x(t, r) = sum_alpha f_alpha(t) sum_l g_{alpha,l}(r) 4 pi Y_l0(z^) Y_l0(r^),
the six f_alpha = sin(O_k t) (paired with even l) and cos(O_k t) (odd l), O_k in {w, w + W, w - W},
  g = (E0/w) w_k (-1)^{l/2} j_l(O_k r / c)          (sin, l even),
  g = -(E0/w) w_k (-1)^{(l-1)/2} j_l(O_k r / c)     (cos, l odd),   w_k = (1/2, -1/4, -1/4).
Reading: the six functions are on for 0 < t < T (the window's retardation z/c, at most r_max / c,
is neglected).

Coupling (same sign convention as the dipole operator: H_I = -c alpha_x A_x). Between the row basis
function i of channel (kappa', mu') and the column function j of channel (kappa, mu),
  <psi_i| alpha_x A_x |psi_j> = i sum_alpha f_alpha sum_l [ Ht_l(kappa, kappa', mu, mu') int P_i(kappa') Q_j(kappa) g
                                                           - Ht_l(kappa', kappa, mu', mu) int Q_i(kappa') P_j(kappa) g ],
  Ht_l(k1, k2, m1, m2) = 4 pi Y_l0(z^) <X_{-k1, m1}| sigma_x Y_l0 |X_{k2, m2}>   (eq. Htheta),
which is Hermitian; the radial integrals are bilinear in (kappa', kappa) (the DKB functions are
linear in kappa), four pieces kappa'^a kappa^b each (eq. fullH).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.sparse as sp
from scipy.special import spherical_jn

from .desc import CouplingTerm, OperatorDesc, Pulse, Workload
from . import dkb


def _fact(n: int) -> int:
    return math.factorial(n)


def wigner_3j(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int) -> float:
    """Wigner 3j symbol for integer arguments (Racah's formula, exact integer sums)."""
    if m1 + m2 + m3 != 0 or not (abs(j1 - j2) <= j3 <= j1 + j2):
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    tri = Fraction(_fact(j1 + j2 - j3) * _fact(j1 - j2 + j3) * _fact(-j1 + j2 + j3), _fact(j1 + j2 + j3 + 1))
    pre = tri * _fact(j1 + m1) * _fact(j1 - m1) * _fact(j2 + m2) * _fact(j2 - m2) * _fact(j3 + m3) * _fact(j3 - m3)
    s = Fraction(0)
    for k in range(max(0, j2 - j3 - m1, j1 - j3 + m2), min(j1 + j2 - j3, j1 - m1, j2 + m2) + 1):
        s += Fraction((-1) ** k, _fact(k) * _fact(j1 + j2 - j3 - k) * _fact(j1 - m1 - k) * _fact(j2 + m2 - k)
                      * _fact(j3 - j2 + m1 + k) * _fact(j3 - j1 - m2 + k))
    val = float(s) * math.sqrt(float(pre))
    return (-1) ** (j1 - j2 - m3) * val


def gaunt(l1: int, m1: int, l: int, l2: int, m2: int) -> float:
    """int conj(Y_{l1 m1}) Y_{l 0} Y_{l2 m2} dOmega (eq. GauntCoef with conj(Y_{l1 m1}) = (-1)^m1 Y_{l1,-m1})."""
    if m1 != m2:
        return 0.0
    return (-1) ** m1 * math.sqrt((2 * l1 + 1) * (2 * l + 1) * (2 * l2 + 1) / (4 * math.pi)) * \
        wigner_3j(l1, l, l2, 0, 0, 0) * wigner_3j(l1, l, l2, -m1, 0, m2)


def h_theta(l: int, k1: int, m1_2: int, k2: int, m2_2: int) -> float:
    """Ht_l(k1, k2, mu1, mu2) = 4 pi Y_l0(z^) <X_{-k1, mu1}| sigma_x Y_l0 |X_{k2, mu2}> (eq. Htheta), mu = m_2 / 2.

    X_{k, mu} = C1 Y_{l_k, mu-1/2} up + C2 Y_{l_k, mu+1/2} down (eq. spinorbasis); sigma_x swaps the spin
    components, so only mu1 = mu2 +- 1 survive (eq. HthetaExpand)."""
    lb1 = dkb.l_of_kappa(-k1)
    l2 = dkb.l_of_kappa(k2)
    d1, d2 = dkb.clebsch_spin_half(lb1, 2 * abs(k1) - 1, m1_2)
    c1, c2 = dkb.clebsch_spin_half(l2, 2 * abs(k2) - 1, m2_2)
    # up component of X_{-k1} (Y_{lb1, mu1 - 1/2}) meets the down component of X_{k2} (Y_{l2, mu2 + 1/2})
    val = 0.0
    if m1_2 - 1 == m2_2 + 1:
        val += d1 * c2 * gaunt(lb1, (m1_2 - 1) // 2, l, l2, (m2_2 + 1) // 2)
    if m1_2 + 1 == m2_2 - 1:
        val += d2 * c1 * gaunt(lb1, (m1_2 + 1) // 2, l, l2, (m2_2 - 1) // 2)
    return 4 * math.pi * math.sqrt((2 * l + 1) / (4 * math.pi)) * val


def channels(kappa_max: int, mu2_max: int):
    """(kappa, 2 mu) for 1 <= |kappa| <= kappa_max, |mu| < |kappa|, |mu| <= mu2_max / 2, ordered by
    (l, j) and then mu (the order of the synthetic beyond-dipole recipe)."""
    out = []
    for k in dkb.kappa_list_by_l(kappa_max):
        if abs(k) > kappa_max:
            continue
        for m2 in range(-mu2_max, mu2_max + 1, 2):
            if abs(m2) < 2 * abs(k):
                out.append((k, m2))
    return out


def angular_matrix(l: int, chans) -> sp.csr_matrix:
    """A[j'][j] = Ht_l(kappa_j, kappa_j', mu_j, mu_j'): the angular factor of the first coupling in the
    module docstring (output channel j', input channel j)."""
    n = len(chans)
    rows, cols, vals = [], [], []
    for jp, (kp, mp) in enumerate(chans):
        for j, (k, m) in enumerate(chans):
            if abs(mp - m) != 2:
                continue
            v = h_theta(l, k, m, kp, mp)
            if v != 0.0:
                rows.append(jp); cols.append(j); vals.append(v)
    a = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    a.sort_indices()
    return a


def angular_matrix_2(l: int, chans) -> sp.csr_matrix:
    """B[j'][j] = Ht_l(kappa_j', kappa_j, mu_j', mu_j) (the second coupling of the docstring)."""
    n = len(chans)
    rows, cols, vals = [], [], []
    for jp, (kp, mp) in enumerate(chans):
        for j, (k, m) in enumerate(chans):
            if abs(mp - m) != 2:
                continue
            v = h_theta(l, kp, mp, k, m)
            if v != 0.0:
                rows.append(jp); cols.append(j); vals.append(v)
    b = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    b.sort_indices()
    return b


def time_functions(omega: float, T: float):
    """The six f_alpha (eq. bdpA) as unit-amplitude carriers on (0, T), and for each its (O_k, w_k,
    kind) with kind 0 = sin(O t) (even l), 1 = cos(O t) (odd l)."""
    W = 2 * math.pi / T
    fs, meta = [], []
    for Om, wk in ((omega, 0.5), (omega + W, -0.25), (omega - W, -0.25)):
        fs.append(Pulse(1.0, T, Om, 0.0, False))            # sin(O t)
        meta.append((Om, wk, 0))
        fs.append(Pulse(1.0, T, Om, math.pi / 2, False))    # cos(O t)
        meta.append((Om, wk, 1))
    return fs, meta


def radial_weight(l: int, Om: float, wk: float, kind: int, E0: float, omega: float, r: np.ndarray, c: float):
    """g_{alpha,l}(r) of eq. bdpA (zero when the parity of l does not match the kind)."""
    if (kind == 0 and l % 2) or (kind == 1 and l % 2 == 0):
        return None
    sign = (-1) ** (l // 2) if kind == 0 else -((-1) ** ((l - 1) // 2))
    return (E0 / omega) * wk * sign * spherical_jn(l, Om * r / c)


def coupling_terms(basis, chans, l_max: int, E0: float, omega: float, T: float, c: float = dkb.C_LIGHT):
    """Coupling terms of H_I = -c alpha_x A_x in the library's form (K^a A K^b) (x) R, coef, field."""
    nr = basis.nr
    hb = basis.order - 1
    comp = dkb.dkb_components(basis, c)
    fs, meta = time_functions(omega, T)
    r = basis.r
    terms = []
    for l in range(l_max + 1):
        A1 = angular_matrix(l, chans)
        A2 = angular_matrix_2(l, chans)
        if A1.nnz == 0 and A2.nnz == 0:
            continue
        for fi, (Om, wk, kind) in enumerate(meta):
            g = radial_weight(l, Om, wk, kind, E0, omega, r, c)
            if g is None:
                continue
            gw = g[:, None]
            for a in (0, 1):
                for b in (0, 1):
                    R1 = np.zeros((2, 2, 2 * hb + 1, nr))
                    R2 = np.zeros((2, 2, 2 * hb + 1, nr))
                    for sr in (0, 1):
                        for sc in (0, 1):
                            # int P_row(kappa')^a-piece Q_col(kappa)^b-piece g dr, and Q_row P_col
                            R1[sr, sc] = basis.band_integral(comp[sr]["P"][a] * gw, comp[sc]["Q"][b])
                            R2[sr, sc] = basis.band_integral(comp[sr]["Q"][a] * gw, comp[sc]["P"][b])
                    if A1.nnz and np.any(R1):
                        terms.append(CouplingTerm(A1.indptr.astype(np.int32), A1.indices.astype(np.int32),
                                                  A1.data.copy(), R1, (a, b), complex(0.0, -c), fi))
                    if A2.nnz and np.any(R2):
                        terms.append(CouplingTerm(A2.indptr.astype(np.int32), A2.indices.astype(np.int32),
                                                  A2.data.copy(), R2, (a, b), complex(0.0, c), fi))
    return terms, fs


def hydrogen_beyond_dipole(nr: int = 300, r_max: float = 60.0, kappa_max: int = 4, mu2_max: int = 3, l_max: int = 3,
                           E0: float = 1.0, omega: float = 1.0, cycles: int = 2, Z: float = 1.0,
                           c: float = dkb.C_LIGHT):
    """Hydrogen in the beyond-dipole pulse: OperatorDesc with the six time functions of eq. bdpA,
    the channel list, the radial basis and the pulses (one instance)."""
    n_int = nr + 3 - (dkb.ORDER - 1)
    br = dkb.lin_exp_breakpoints(n_int, r_max)
    basis = dkb.RadialBasis(br)
    assert basis.nr == nr
    h_poly, s_poly, _ = dkb.dirac_radial_matrices(basis, Z, c)
    chans = channels(kappa_max, mu2_max)
    T = cycles * 2 * math.pi / omega
    terms, fs = coupling_terms(basis, chans, l_max, E0, omega, T, c)
    op = OperatorDesc(nr=nr, nang=len(chans), hb=dkb.HB, kappa=np.array([k for k, _ in chans], dtype=np.float64),
                      h_poly=h_poly, s_poly=s_poly, terms=terms, n_fields=len(fs))
    return op, chans, basis, fs, T


def workload(nr: int = 300, r_max: float = 60.0, kappa_max: int = 4, mu2_max: int = 3, l_max: int = 3,
             E0: float = 1.0, omega: float = 1.0, cycles: int = 2, dt: float = 4e-3, t0_frac: float = 0.25,
             n_steps: int = 20):
    """One instance: the hydrogen ground state (kappa = -1, mu = 1/2) in the beyond-dipole pulse,
    started at t0 = t0_frac * T (the coupling switched on)."""
    op, chans, basis, fs, T = hydrogen_beyond_dipole(nr, r_max, kappa_max, mu2_max, l_max, E0, omega, cycles)
    j0 = chans.index((-1, 1))
    w, v = dkb.bound_states(op.h_poly, op.s_poly, -1.0, nr, op.hb, n_states=1)
    S = dkb.sparse_block(op.s_poly, -1.0, nr, op.hb)
    vec = v[:, 0] / math.sqrt(v[:, 0] @ (S @ v[:, 0]))
    psi0 = np.zeros((1, op.nang, 2, nr), dtype=np.complex128)
    psi0[0, j0, 0] = vec[:nr]
    psi0[0, j0, 1] = vec[nr:]
    return Workload("beyond", op, psi0, [fs], dt=dt, t0=t0_frac * T, n_steps=np.array([n_steps], dtype=np.int32),
                    tol=1e-12, meta={"T": T, "E_ground": float(w[0]), "kappa_max": kappa_max, "mu2_max": mu2_max,
                                     "l_max": l_max, "E0": E0, "omega": omega})
