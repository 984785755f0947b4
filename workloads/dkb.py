"""Hydrogen-like Dirac operator in a dual-kinetic-balance B-spline basis (input generator).

Produces the kappa-polynomial radial matrices of paper eq. fullH for a field-free H0
and overlap S, and the velocity-gauge dipole coupling, in the band format of
``workloads.desc``. It is setup work done once before time propagation (paper
Sec. 3.1, step 1a); the time step itself never appears here.

Readings of points the paper leaves open (each one is listed in the design notes):
  * radial operator (with p = -i grad, standard alpha, shifted beta of Sec. 2.1):
        H_kappa = [[V, c(-d/dr + kappa/r)], [c(d/dr + kappa/r), V - 2c^2]],  V = -Z/r,
    with psi = r^-1 (P X_{kappa mu}, i Q X_{-kappa mu}) (eq. basis). The kinetic part is
    integrated in the symmetric form (integration by parts, boundary terms vanish).
  * DKB basis (eq. dualkinetic): k <= N: (u, (u' + kappa u/r)/2c); k > N: ((u' - kappa u/r)/2c, u).
  * B-splines of order 7 (degree 6) by the de Boor recursion of Sec. 2.2 on a knot vector
    padded to multiplicity 7 at both ends. At r = 0 only the spline that is nonzero there is
    dropped: the next one (linear at the origin) is needed for s1/2 states, whose large
    component starts linearly (dropping it too leaves a 2e-3 error on the 1s energy). At
    r_max the last two splines are dropped, so every kept function and its derivative
    vanish there and the symmetric kinetic form is exact.
  * every B-spline is scaled to unit L2 norm (kappa-independent diagonal rescaling; it
    improves the conditioning of S without changing the physics).
  * linear-exponential breakpoints: spacing h_q = min(h_min * g^q, h_lin), h_lin set so
    the last breakpoint is r_max.
  * Gauss-Legendre quadrature with order + 3 points per knot interval.
  * dipole coupling H_I = -c A(t) alpha_z at fixed mu (quantisation axis along the
    polarisation); angular factor <X_{kappa' mu}|sigma_z|X_{-kappa mu}> from
    Clebsch-Gordan coefficients; radial factor int P_{kappa'} Q_{kappa} dr, bilinear in
    (kappa', kappa) as in eq. fullH.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .desc import C_LIGHT, CouplingTerm, OperatorDesc, Pulse, Workload
from .synthetic import band_transpose, kappa_list_by_l, l_of_kappa

ORDER = 7
HB = ORDER - 1


def lin_exp_breakpoints(n_int: int, r_max: float, h_min: float = 1e-2, growth: float = 1.05) -> np.ndarray:
    """n_int + 1 breakpoints on [0, r_max]: geometric growth from h_min, then uniform."""
    def total(h_lin):
        h = np.minimum(h_min * growth ** np.arange(n_int), h_lin)
        return h.sum(), h
    lo, hi = h_min, r_max
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s, _ = total(mid)
        if s < r_max:
            lo = mid
        else:
            hi = mid
    _, h = total(0.5 * (lo + hi))
    br = np.concatenate([[0.0], np.cumsum(h)])
    br *= r_max / br[-1]
    return br


def knot_vector(breakpoints: np.ndarray, order: int = ORDER) -> np.ndarray:
    return np.concatenate([np.full(order - 1, breakpoints[0]), breakpoints, np.full(order - 1, breakpoints[-1])])


def _local_bsplines(t: np.ndarray, order: int, mu: np.ndarray, x: np.ndarray):
    """Values of the `order` B-splines nonzero on knot interval mu at points x (de Boor recursion).

    Returns a list vals[q] for q = 1..order, vals[q] of shape [P, q]: vals[q][:, r] is
    B_{mu-q+1+r, q}(x) (order-q spline, degree q-1).
    """
    P = x.shape[0]
    vals = [None, np.ones((P, 1))]
    for q in range(2, order + 1):
        prev = vals[q - 1]
        cur = np.zeros((P, q))
        for r in range(q):
            i = mu - q + 1 + r
            if r >= 1:  # left term uses B_{i, q-1} = prev[:, r-1]
                den = t[i + q - 1] - t[i]
                safe = np.where(den > 0, den, 1.0)
                cur[:, r] += np.where(den > 0, (x - t[i]) / safe, 0.0) * prev[:, r - 1]
            if r <= q - 2:  # right term uses B_{i+1, q-1} = prev[:, r]
                den = t[i + q] - t[i + 1]
                safe = np.where(den > 0, den, 1.0)
                cur[:, r] += np.where(den > 0, (t[i + q] - x) / safe, 0.0) * prev[:, r]
        vals.append(cur)
    return vals


def _deriv(t, q, mu, prev):
    """Derivative of the order-q splines on interval mu from the order-(q-1) local array prev [P, q-1]."""
    P = prev.shape[0]
    out = np.zeros((P, q))
    for r in range(q):
        i = mu - q + 1 + r
        if r >= 1:
            den = t[i + q - 1] - t[i]
            out[:, r] += np.where(den > 0, 1.0 / np.where(den > 0, den, 1.0), 0.0) * prev[:, r - 1]
        if r <= q - 2:
            den = t[i + q] - t[i + 1]
            out[:, r] -= np.where(den > 0, 1.0 / np.where(den > 0, den, 1.0), 0.0) * prev[:, r]
    return (q - 1) * out


class RadialBasis:
    """Order-7 B-splines on a breakpoint grid, evaluated at Gauss-Legendre points.

    Attributes: r [Q], w [Q] (points/weights), first [Q] (global index of the first local
    spline), u, du, d2u [Q, order] (unit-L2-normalised values and derivatives), nr (kept
    functions), drop_lo = 1 (global index of basis function 0).
    """

    def __init__(self, breakpoints: np.ndarray, order: int = ORDER, n_gauss: int | None = None):
        self.order = order
        self.breakpoints = breakpoints
        t = knot_vector(breakpoints, order)
        self.t = t
        n_int = len(breakpoints) - 1
        n_spl = n_int + order - 1
        ng = n_gauss or order + 3
        gx, gw = np.polynomial.legendre.leggauss(ng)
        a, b = breakpoints[:-1], breakpoints[1:]
        r = (0.5 * (b - a)[:, None] * gx[None, :] + 0.5 * (a + b)[:, None]).ravel()
        w = (0.5 * (b - a)[:, None] * gw[None, :]).ravel()
        qidx = np.repeat(np.arange(n_int), ng)
        mu = qidx + order - 1
        vals = _local_bsplines(t, order, mu, r)
        u = vals[order]
        du = _deriv(t, order, mu, vals[order - 1])
        d2u = _deriv(t, order, mu, _deriv(t, order - 1, mu, vals[order - 2]))
        first = qidx  # global index of local spline 0 on interval q is q
        self.drop_lo, self.drop_hi = 1, 2
        self.n_spl = n_spl
        self.nr = n_spl - self.drop_lo - self.drop_hi
        # unit L2 normalisation of every spline
        norm2 = np.zeros(n_spl)
        np.add.at(norm2, (first[:, None] + np.arange(order)[None, :]).ravel(), (w[:, None] * u * u).ravel())
        scale = 1.0 / np.sqrt(np.where(norm2 > 0, norm2, 1.0))
        sc = scale[first[:, None] + np.arange(order)[None, :]]
        self.r, self.w, self.first = r, w, first
        self.u, self.du, self.d2u = u * sc, du * sc, d2u * sc

    def band_integral(self, f_row, f_col):
        """Banded matrix M[i][i'] = int f_row_i(r) f_col_i'(r) dr over kept basis functions.

        f_row, f_col: [Q, order] arrays of the local functions. Returns band[d+hb][i].
        """
        order, hb = self.order, self.order - 1
        band = np.zeros((2 * hb + 1, self.nr))
        for a in range(order):
            ia = self.first + a - self.drop_lo
            for b in range(order):
                ib = self.first + b - self.drop_lo
                ok = (ia >= 0) & (ia < self.nr) & (ib >= 0) & (ib < self.nr)
                np.add.at(band, (ib[ok] - ia[ok] + hb, ia[ok]), (self.w * f_row[:, a] * f_col[:, b])[ok])
        return band


def dkb_components(basis: RadialBasis, c: float):
    """Per spinor type s the kappa-linear local functions P, Q and dP/dr: each a pair (x0, x1)."""
    u, du, d2u = basis.u, basis.du, basis.d2u
    r = basis.r[:, None]
    z = np.zeros_like(u)
    comp = {}
    # s = 0: P = u, Q = (u' + kappa u / r) / 2c
    comp[0] = dict(P=(u, z), Q=(du / (2 * c), u / (2 * c * r)), dP=(du, z))
    # s = 1: P = (u' - kappa u / r) / 2c, Q = u
    comp[1] = dict(P=(du / (2 * c), -u / (2 * c * r)), Q=(u, z),
                   dP=(d2u / (2 * c), -(du / r - u / (r * r)) / (2 * c)))
    return comp


def dirac_radial_matrices(basis: RadialBasis, Z: float = 1.0, c: float = C_LIGHT):
    """kappa-polynomial bands h_poly [4][2][2][2hb+1][nr] and s_poly [3][2][2][2hb+1][nr] of the
    radial Dirac operator and overlap, plus the dipole radial pieces g[(a, b)] [2][2][2hb+1][nr]
    (a = exponent of the row kappa, b = exponent of the column kappa)."""
    hb = basis.order - 1
    nr = basis.nr
    r = basis.r[:, None, None]
    V = -Z / r
    comp = dkb_components(basis, c)
    h_poly = np.zeros((4, 2, 2, 2 * hb + 1, nr))
    s_poly = np.zeros((3, 2, 2, 2 * hb + 1, nr))
    g = {(a, b): np.zeros((2, 2, 2 * hb + 1, nr)) for a in (0, 1) for b in (0, 1)}
    for sr in (0, 1):
        A = comp[sr]
        for sc in (0, 1):
            B = comp[sc]
            PP, QQ = _pmul(A["P"], B["P"]), _pmul(A["Q"], B["Q"])
            dPQ, QdP = _pmul(A["dP"], B["Q"]), _pmul(A["Q"], B["dP"])
            PQ, QP = _pmul(A["P"], B["Q"]), _pmul(A["Q"], B["P"])
            # overlap: P_a P_b + Q_a Q_b (kappa-quadratic)
            # Hamiltonian: V (PP + QQ) - 2c^2 QQ + c (dP_a Q_b + Q_a dP_b) + c kappa (P_a Q_b + Q_a P_b) / r
            hcoef = [0.0] * 4
            for n in range(3):
                s_poly[n, sr, sc] = _band_of_products(basis, PP[n] + QQ[n])
                hcoef[n] = hcoef[n] + V * (PP[n] + QQ[n]) - 2 * c * c * QQ[n] + c * (dPQ[n] + QdP[n])
                hcoef[n + 1] = hcoef[n + 1] + c * (PQ[n] + QP[n]) / r
            for n in range(4):
                h_poly[n, sr, sc] = _band_of_products(basis, hcoef[n])
            # dipole radial factor int P_{row}(kappa') Q_{col}(kappa) dr
            g[(0, 0)][sr, sc] = basis.band_integral(A["P"][0], B["Q"][0])
            g[(1, 0)][sr, sc] = basis.band_integral(A["P"][1], B["Q"][0])
            g[(0, 1)][sr, sc] = basis.band_integral(A["P"][0], B["Q"][1])
            g[(1, 1)][sr, sc] = basis.band_integral(A["P"][1], B["Q"][1])
    return h_poly, s_poly, g


def _band_of_products(basis, prod):
    """prod[Q, a, b] (local row a, column b) -> band; prod given as per-point outer products."""
    order, hb = basis.order, basis.order - 1
    band = np.zeros((2 * hb + 1, basis.nr))
    for a in range(order):
        ia = basis.first + a - basis.drop_lo
        for b in range(order):
            ib = basis.first + b - basis.drop_lo
            ok = (ia >= 0) & (ia < basis.nr) & (ib >= 0) & (ib < basis.nr)
            np.add.at(band, (ib[ok] - ia[ok] + hb, ia[ok]), (basis.w * prod[:, a, b])[ok])
    return band


def _pmul(f, g):
    """(f0 + k f1)(g0 + k g1) for local functions f, g [Q, order] -> 3 kappa coefficients, each the
    per-point outer product [Q, order(row), order(col)]."""
    return [f[0][:, :, None] * g[0][:, None, :],
            f[0][:, :, None] * g[1][:, None, :] + f[1][:, :, None] * g[0][:, None, :],
            f[1][:, :, None] * g[1][:, None, :]]


def clebsch_spin_half(l: int, j2: int, mu2: int):
    """(C1, C2): <l, mu-1/2; 1/2, 1/2 | j mu> and <l, mu+1/2; 1/2, -1/2 | j mu> (Condon-Shortley),
    with j = j2/2, mu = mu2/2 (closed forms for coupling with spin 1/2)."""
    mu = mu2 / 2.0
    den = 2 * l + 1
    if j2 == 2 * l + 1:  # j = l + 1/2
        c1 = math.sqrt(max(l + mu + 0.5, 0.0) / den)
        c2 = math.sqrt(max(l - mu + 0.5, 0.0) / den)
    elif j2 == 2 * l - 1:  # j = l - 1/2
        c1 = -math.sqrt(max(l - mu + 0.5, 0.0) / den)
        c2 = math.sqrt(max(l + mu + 0.5, 0.0) / den)
    else:
        raise ValueError("j must be l +- 1/2")
    # components whose |m_l| exceeds l vanish
    if abs(mu - 0.5) > l:
        c1 = 0.0
    if abs(mu + 0.5) > l:
        c2 = 0.0
    return c1, c2


def sigma_z_angular(kp: int, k: int, mu2: int) -> float:
    """<X_{kp, mu}| sigma_z |X_{k, mu}>: nonzero only when l_kp == l_k."""
    if l_of_kappa(kp) != l_of_kappa(k):
        return 0.0
    l = l_of_kappa(k)
    a1, a2 = clebsch_spin_half(l, 2 * abs(kp) - 1, mu2)
    b1, b2 = clebsch_spin_half(l, 2 * abs(k) - 1, mu2)
    return a1 * b1 - a2 * b2


def dipole_terms(kappas, mu2: int, g, nr: int, c: float = C_LIGHT):
    """Coupling terms of H_I = -c A(t) alpha_z (field index 0 is A(t)).

    Matrix element between (kappa', s', i') and (kappa, s, i):
      -i c A(t) [ Th(kappa', -kappa) W(kappa', kappa) - Th(kappa, -kappa') W(kappa, kappa')^T ],
    W(kappa', kappa) = sum_{a,b} kappa'^a kappa^b g[(a, b)], Th(x, y) = <X_x|sigma_z|X_y>.
    """
    n = len(kappas)
    th = np.zeros((n, n))
    for jp, kp in enumerate(kappas):
        for j, k in enumerate(kappas):
            th[jp, j] = sigma_z_angular(kp, -k, mu2)
    a1 = sp.csr_matrix(th)
    a1.eliminate_zeros(); a1.sort_indices()
    a2 = sp.csr_matrix(th.T)
    a2.eliminate_zeros(); a2.sort_indices()
    terms = []
    hb = g[(0, 0)].shape[2] // 2
    for (a, b), gab in g.items():
        terms.append(CouplingTerm(a1.indptr.astype(np.int32), a1.indices.astype(np.int32), a1.data.copy(),
                                  gab.copy(), (a, b), complex(0.0, -c), 0))
        gt = np.zeros_like(gab)
        for sr in (0, 1):
            for sc in (0, 1):
                gt[sr, sc] = band_transpose(gab[sc, sr], nr, hb)
        terms.append(CouplingTerm(a2.indptr.astype(np.int32), a2.indices.astype(np.int32), a2.data.copy(),
                                  gt, (b, a), complex(0.0, c), 0))
    return terms, th


def dense_block(h_poly, kappa, nr, hb):
    """Dense 2nr x 2nr matrix sum_n kappa^n h_poly[n] (generator-side helper for eigenstates)."""
    out = np.zeros((2 * nr, 2 * nr))
    idx = np.arange(nr)
    for n in range(h_poly.shape[0]):
        kn = kappa ** n
        for s in range(2):
            for s2 in range(2):
                for d in range(-hb, hb + 1):
                    ok = (idx + d >= 0) & (idx + d < nr)
                    out[s * nr + idx[ok], s2 * nr + idx[ok] + d] += kn * h_poly[n, s, s2, d + hb, ok]
    return out


def sparse_block(h_poly, kappa, nr, hb):
    rows, cols, vals = [], [], []
    idx = np.arange(nr)
    for s in range(2):
        for s2 in range(2):
            for d in range(-hb, hb + 1):
                ok = (idx + d >= 0) & (idx + d < nr)
                v = sum(kappa ** n * h_poly[n, s, s2, d + hb, ok] for n in range(h_poly.shape[0]))
                rows.append(s * nr + idx[ok]); cols.append(s2 * nr + idx[ok] + d); vals.append(v)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(2 * nr, 2 * nr))


def bound_states(h_poly, s_poly, kappa, nr, hb, n_states=3, c=C_LIGHT, sigma=None):
    """Lowest generalised eigenpairs above -c^2 of the kappa block (shift-invert near sigma)."""
    H = sparse_block(h_poly, kappa, nr, hb)
    S = sparse_block(s_poly, kappa, nr, hb)
    if 2 * nr <= 1600:
        w, v = sla.eigh(H.toarray(), S.toarray())
    else:
        sig = -0.6 if sigma is None else sigma
        w, v = spla.eigsh(H.tocsc(), k=n_states + 4, M=S.tocsc(), sigma=sig, which="LM")
        order = np.argsort(w)
        w, v = w[order], v[:, order]
    keep = w > -c * c
    return w[keep][:n_states], v[:, keep][:, :n_states]


def hydrogen_operator(nr: int = 2000, r_max: float = 200.0, lmax: int = 20, mu2: int = 1, Z: float = 1.0,
                      c: float = C_LIGHT, h_min: float = 1e-2, growth: float = 1.05):
    """Field-free H0, S and dipole coupling of hydrogen on nr DKB radial pairs, channels l <= lmax at mu."""
    n_int = nr + 3 - (ORDER - 1)
    br = lin_exp_breakpoints(n_int, r_max, h_min, growth)
    basis = RadialBasis(br)
    assert basis.nr == nr
    h_poly, s_poly, g = dirac_radial_matrices(basis, Z, c)
    kappas = [k for k in kappa_list_by_l(lmax) if abs(mu2) < 2 * abs(k)]
    terms, th = dipole_terms(kappas, mu2, g, nr, c)
    op = OperatorDesc(nr=nr, nang=len(kappas), hb=HB, kappa=np.array(kappas, dtype=np.float64),
                      h_poly=h_poly, s_poly=s_poly, terms=terms, n_fields=1)
    return op, basis, th


def config2(nr: int = 2000, r_max: float = 200.0, lmax: int = 20, E0: float = 0.05, omega: float = 0.057,
            cycles: int = 8, dt: float = 2e-4, n_steps: int = 2000, driven: bool = False) -> Workload:
    """Hydrogen dipole case: ground state, sin^2 pulse A(t) = (E0/w) sin^2(pi t/T) sin(w t)."""
    op, basis, _ = hydrogen_operator(nr, r_max, lmax)
    T = cycles * 2 * math.pi / omega
    j0 = int(np.nonzero(op.kappa == -1)[0][0])
    w, v = bound_states(op.h_poly, op.s_poly, -1.0, nr, op.hb, n_states=1)
    psi0 = np.zeros((1, op.nang, 2, nr), dtype=np.complex128)
    vec = v[:, 0]
    S = sparse_block(op.s_poly, -1.0, nr, op.hb)
    vec = vec / math.sqrt(vec @ (S @ vec))
    if vec[np.argmax(np.abs(vec))] < 0:
        vec = -vec
    psi0[0, j0, 0] = vec[:nr]
    psi0[0, j0, 1] = vec[nr:]
    t0 = (T / 2 + math.pi / (2 * omega)) if driven else 0.0
    pulse = Pulse(amp=E0 / omega, T=T, omega=omega, phase=0.0, envelope=True)
    return Workload("c2d" if driven else "c2", op, psi0, [[pulse]], dt=dt, t0=t0,
                    n_steps=np.array([n_steps], dtype=np.int32), tol=1e-12,
                    meta={"E_ground": float(w[0]), "r_max": r_max, "lmax": lmax, "E0": E0})


