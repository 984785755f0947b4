"""Seeded synthetic operators with the block-banded structure of the paper's Hamiltonian.

These are input generators only. They draw random numbers with
``numpy.random.default_rng(seed)`` (PCG64) in a fixed order and return
``Workload`` objects; neither the GPU path nor the oracle re-draws anything.

Structure follows paper Sec. 2.2: per-channel radial blocks banded with the
B-spline half-bandwidth (order 7 -> 6 neighbours on each side), a -2c^2 offset on
the small (Q-type) component (shifted beta of Sec. 2.1), and coupling terms that are
Kronecker products of a sparse angular matrix and a banded radial matrix (eq. fullH).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .desc import C_LIGHT, CouplingTerm, OperatorDesc, Pulse, Workload

HB = 6  # half-bandwidth of order-7 B-spline radial matrices


def l_of_kappa(k: int) -> int:
    """Orbital angular momentum of the large component: l = k for k > 0, -k-1 for k < 0."""
    return k if k > 0 else -k - 1


def kappa_list_by_l(lmax: int):
    """All kappa with l_kappa <= lmax ordered by (l, j): kappa = l (j = l-1/2) then -(l+1)."""
    out = []
    for l in range(lmax + 1):
        if l >= 1:
            out.append(l)
        out.append(-(l + 1))
    return out


def _herm_band_complex(rng, nr, hb, diag):
    """Complex Hermitian banded block as band[d+hb][i]; off-diagonals Re, Im ~ N(0,1)/10."""
    up = (rng.standard_normal((hb, nr)) + 1j * rng.standard_normal((hb, nr))) / 10.0
    band = np.zeros((2 * hb + 1, nr), dtype=np.complex128)
    band[hb] = diag
    idx = np.arange(nr)
    for d in range(1, hb + 1):
        valid = idx + d < nr
        band[hb + d][valid] = up[d - 1][valid]  # entry (i, i+d)
        lower = idx - d >= 0
        band[hb - d][lower] = np.conj(up[d - 1][idx[lower] - d])  # entry (i, i-d) = conj((i-d, i))
    return band


def _sym_band_real(rng, nr, hb, scale=0.1, diag=None):
    """Real symmetric banded matrix as band[d+hb][i]; entries (i, i+d), d = 0..hb, ~ N(0,1)*scale."""
    lo = rng.standard_normal((hb + 1, nr)) * scale
    band = np.zeros((2 * hb + 1, nr))
    idx = np.arange(nr)
    band[hb] = lo[0] if diag is None else diag
    for d in range(1, hb + 1):
        valid = idx + d < nr
        band[hb + d][valid] = lo[d][valid]
        lower = idx - d >= 0
        band[hb - d][lower] = lo[d][idx[lower] - d]
    return band


def band_to_sparse(band, nr, hb):
    """Real or complex band[d+hb][i] -> scipy CSR (only used for generator-side scaling)."""
    rows, cols, vals = [], [], []
    idx = np.arange(nr)
    for d in range(-hb, hb + 1):
        ok = (idx + d >= 0) & (idx + d < nr)
        rows.append(idx[ok]); cols.append(idx[ok] + d); vals.append(band[d + hb][ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nr, nr))


def _spectral_norm_sym(m) -> float:
    """Largest |eigenvalue| of a real symmetric sparse matrix (deterministic start vector)."""
    n = m.shape[0]
    v0 = np.ones(n) / math.sqrt(n)
    if n <= 64:
        return float(np.max(np.abs(np.linalg.eigvalsh(m.toarray()))))
    w = spla.eigsh(m, k=1, which="LM", v0=v0, return_eigenvectors=False, tol=1e-12)
    return float(abs(w[0]))


def _random_state(rng, batch, nang, nr):
    psi = rng.standard_normal((nang, 2, nr)) + 1j * rng.standard_normal((nang, 2, nr))
    psi /= np.linalg.norm(psi)
    return np.repeat(psi[None], batch, axis=0)


def _tridiag_channels(nang):
    """A_1 links channel j with j+-1 with weight 1/sqrt(2)."""
    rows, cols = [], []
    for j in range(nang):
        for jj in (j - 1, j + 1):
            if 0 <= jj < nang:
                rows.append(j); cols.append(jj)
    a = sp.csr_matrix((np.full(len(rows), 1 / math.sqrt(2)), (rows, cols)), shape=(nang, nang))
    a.sort_indices()
    return a


def _csr_fields(a):
    a = sp.csr_matrix(a)
    a.sort_indices()
    return a.indptr.astype(np.int32), a.indices.astype(np.int32), a.data.astype(np.float64)


def _identity_s(r_band_1):
    rb = np.zeros((2, 2) + r_band_1.shape)
    rb[0, 0] = r_band_1
    rb[1, 1] = r_band_1
    return rb


def block_banded_operator(nr: int, nang: int, seed: int, c: float = C_LIGHT):
    """Config-1 recipe: per-channel complex Hermitian H0 blocks, S = I, one coupling term.

    Draw order: H0 blocks (j-major, then s), R_1, then the initial state.
    Returns (OperatorDesc, psi0 [nang][2][nr], rng after the draws).
    """
    rng = np.random.default_rng(seed)
    hb = HB
    h_chan = np.zeros((nang, 2, 2, 2 * hb + 1, nr), dtype=np.complex128)
    base = np.linspace(-0.5, 50.0, nr)
    for j in range(nang):
        for s in range(2):
            diag = base - (2 * c * c if s == 1 else 0.0)
            h_chan[j, s, s] = _herm_band_complex(rng, nr, hb, diag)
    r1 = _sym_band_real(rng, nr, hb)
    rp, ci, va = _csr_fields(_tridiag_channels(nang))
    term = CouplingTerm(rp, ci, va, _identity_s(r1), (0, 0), complex(1.0, 0.0), 0)
    op = OperatorDesc(nr=nr, nang=nang, hb=hb, kappa=np.zeros(nang), h_poly=np.zeros((0, 2, 2, 2 * hb + 1, nr)),
                      s_poly=np.zeros((0, 2, 2, 2 * hb + 1, nr)), terms=[term], n_fields=1, h_chan=h_chan)
    psi0 = _random_state(rng, 1, nang, nr)[0]
    return op, psi0, rng


def config1(seed: int = 0, driven: bool = False) -> Workload:
    """Plain FP64 synthetic block-banded step: Nr=200, Nang=8, N=3200, 20 steps of dt=1e-3."""
    op, psi0, _ = block_banded_operator(200, 8, seed)
    T = 20.0
    pulse = Pulse(amp=0.05, T=T, omega=0.057, phase=math.pi / 2, envelope=True)  # E0 sin^2(pi t/T) cos(w t)
    t0 = T / 4 if driven else 0.0
    return Workload("c1d" if driven else "c1", op, psi0[None], [[pulse]], dt=1e-3, t0=t0,
                    n_steps=np.array([20], dtype=np.int32), tol=1e-12, meta={"seed": seed})


def c3_channels(lmax: int = 40, mu_max2: int = 9):
    """(kappa, 2*mu) for all kappa with l_kappa <= lmax and |mu| <= mu_max2/2, |mu| < |kappa|."""
    ch = []
    for k in kappa_list_by_l(lmax):
        for twomu in range(-mu_max2, mu_max2 + 1, 2):
            if abs(twomu) < 2 * abs(k):
                ch.append((k, twomu))
    return ch


def beyond_dipole_operator(nr: int = 4000, lmax: int = 40, mu_max2: int = 9, n_terms: int = 6,
                           seed: int = 0, c: float = C_LIGHT):
    """Config-3 recipe: kappa-cubic H0 per component, S = I, six terms with |dl| <= 2, mu' = mu +- 1.

    Draw order: h_0 (s = 0, 1), h_1..h_3 (s = 0, 1), then for each term A_m values and R_m,
    then the initial state. A_m and R_m are scaled to unit spectral norm.
    """
    rng = np.random.default_rng(seed)
    hb = HB
    ch = c3_channels(lmax, mu_max2)
    nang = len(ch)
    kappa = np.array([k for k, _ in ch], dtype=np.float64)
    h_poly = np.zeros((4, 2, 2, 2 * hb + 1, nr))
    base = np.linspace(-0.5, 50.0, nr)
    for s in range(2):
        h_poly[0, s, s] = _sym_band_real(rng, nr, hb, diag=base - (2 * c * c if s == 1 else 0.0))
    for n in range(1, 4):
        for s in range(2):
            h_poly[n, s, s] = _sym_band_real(rng, nr, hb, scale=0.1 * (1.0 / 41.0) ** n)
    # angular pattern: |l - l'| <= 2, mu' = mu +- 1 (selection rule of the coupling matrix)
    ls = np.array([l_of_kappa(k) for k, _ in ch])
    mus = np.array([m for _, m in ch])
    pat_r, pat_c = [], []
    for j in range(nang):
        ok = (np.abs(ls - ls[j]) <= 2) & (np.abs(mus - mus[j]) == 2)
        for jj in np.nonzero(ok)[0]:
            if jj > j:
                pat_r.append(j); pat_c.append(int(jj))
    pat_r = np.array(pat_r); pat_c = np.array(pat_c)
    terms = []
    for m in range(n_terms):
        v = rng.standard_normal(len(pat_r))
        a = sp.coo_matrix((np.concatenate([v, v]), (np.concatenate([pat_r, pat_c]), np.concatenate([pat_c, pat_r]))),
                          shape=(nang, nang)).tocsr()
        a = a / _spectral_norm_sym(a)
        rb = _sym_band_real(rng, nr, hb)
        rb = rb / _spectral_norm_sym(band_to_sparse(rb, nr, hb))
        rp, ci, va = _csr_fields(a)
        terms.append(CouplingTerm(rp, ci, va, _identity_s(rb), (0, 0), complex(1.0, 0.0), m))
    op = OperatorDesc(nr=nr, nang=nang, hb=hb, kappa=kappa, h_poly=h_poly, s_poly=np.zeros((0, 2, 2, 2 * hb + 1, nr)),
                      terms=terms, n_fields=n_terms)
    psi0 = _random_state(rng, 1, nang, nr)
    return op, psi0


def config3(seed: int = 0, driven: bool = False, nr: int = 4000, lmax: int = 40, mu_max2: int = 9,
            n_steps: int = 10) -> Workload:
    """Beyond-dipole-shaped single-GPU share: Nr=4000, Nang=770, six coupling terms, 10 steps."""
    op, psi0 = beyond_dipole_operator(nr, lmax, mu_max2, 6, seed)
    E0, w, T = 0.05, 0.057, 20.0
    dw = 2 * math.pi / T
    pulses = []
    for delta in (0.0, dw, -dw):
        pulses.append(Pulse(E0, T, w + delta, math.pi / 2, True))  # cos((w+delta) t)
        pulses.append(Pulse(E0, T, w + delta, 0.0, True))  # sin((w+delta) t)
    t0 = T / 4 if driven else 0.0
    return Workload("c3d" if driven else "c3", op, psi0, [pulses], dt=1e-3, t0=t0,
                    n_steps=np.array([n_steps], dtype=np.int32), tol=1e-12,
                    meta={"seed": seed, "lmax": lmax, "mu_max2": mu_max2})


STEPS_PER_CYCLE = 100


def batched_pulses(seeds, dt: float = 1e-3):
    """Per-instance pulses on the compressed time axis: E0 ~ U[0.05, 0.5], CEP ~ U[0, 2pi),
    cycles ~ U{4..12}; 100 steps per cycle, so n_b = 100 * cycles and T_b = n_b * dt."""
    omega = 2 * math.pi / (STEPS_PER_CYCLE * dt)
    pulses, n_steps = [], []
    for sd in seeds:
        r = np.random.default_rng(int(sd))
        E0 = float(r.uniform(0.05, 0.5))
        phi = float(r.uniform(0.0, 2 * math.pi))
        cycles = int(r.integers(4, 13))
        nb = STEPS_PER_CYCLE * cycles
        pulses.append([Pulse(E0, nb * dt, omega, phi + math.pi / 2, True)])  # E0 sin^2 cos(w t + phi)
        n_steps.append(nb)
    return pulses, np.array(n_steps, dtype=np.int32)


def config5(batch: int = 64, nr: int = 2000, nang: int = 41, seed: int = 0, first_seed: int = 10001,
            seeds=None) -> Workload:
    """Batched sweep: `batch` instances of the config-1 recipe at Nr=2000, Nang=41, uneven lengths."""
    op, psi0, _ = block_banded_operator(nr, nang, seed)
    if seeds is None:
        seeds = range(first_seed, first_seed + batch)
    seeds = list(seeds)
    pulses, n_steps = batched_pulses(seeds)
    psi = np.repeat(psi0[None], len(seeds), axis=0)
    return Workload("c5", op, psi, pulses, dt=1e-3, t0=0.0, n_steps=n_steps, tol=1e-12,
                    meta={"seed": seed, "instance_seeds": seeds})


def tiny(nr: int = 20, nang: int = 3, seed: int = 7, s_identity: bool = True, pq_coupling: bool = True,
         n_terms: int = 2) -> Workload:
    """Tiny general operator exercising every feature (kappa polynomials, P-Q coupling, S != I,
    kappa exponents, complex prefactors, several fields, per-channel complex bands)."""
    rng = np.random.default_rng(seed)
    hb = HB
    kappa = np.array([(-1) ** j * (j // 2 + 1) for j in range(nang)], dtype=np.float64)
    h_poly = np.zeros((3, 2, 2, 2 * hb + 1, nr))
    # Hermitian kappa-polynomial H0 with P-Q coupling: block (s, s') = transpose of (s', s)
    for n in range(3):
        for s in range(2):
            h_poly[n, s, s] = _sym_band_real(rng, nr, hb, scale=0.3)
        if pq_coupling:
            g = rng.standard_normal((2 * hb + 1, nr)) * 0.3
            idx = np.arange(nr)
            for d in range(-hb, hb + 1):
                g[d + hb][(idx + d < 0) | (idx + d >= nr)] = 0.0
            h_poly[n, 0, 1] = g
            h_poly[n, 1, 0] = _band_transpose(g, nr, hb)
    h_poly[0, 1, 1, hb] -= 2.0  # small-component offset
    h_chan = np.zeros((nang, 2, 2, 2 * hb + 1, nr), dtype=np.complex128)
    for j in range(nang):
        for s in range(2):
            h_chan[j, s, s] = _herm_band_complex(rng, nr, hb, np.zeros(nr)) * 0.5
    if s_identity:
        s_poly = np.zeros((0, 2, 2, 2 * hb + 1, nr))
    else:
        s_poly = np.zeros((2, 2, 2, 2 * hb + 1, nr))
        for s in range(2):
            s_poly[0, s, s] = _sym_band_real(rng, nr, hb, scale=0.05, diag=np.full(nr, 1.0))
            s_poly[1, s, s] = _sym_band_real(rng, nr, hb, scale=0.01, diag=np.full(nr, 0.02))
    terms = []
    for m in range(n_terms):
        a = sp.random(nang, nang, density=0.6, random_state=int(rng.integers(1 << 30)), format="csr")
        a.data = rng.standard_normal(a.nnz)
        rb = rng.standard_normal((2, 2, 2 * hb + 1, nr)) * 0.2
        idx = np.arange(nr)
        for d in range(-hb, hb + 1):
            rb[:, :, d + hb, (idx + d < 0) | (idx + d >= nr)] = 0.0
        kp = (m % 2, (m // 2) % 2)
        coef = complex(0.0, 1.0) if m % 2 == 0 else complex(0.7, -0.2)
        rp, ci, va = _csr_fields(a)
        terms.append(CouplingTerm(rp, ci, va, rb, kp, coef, m % 2))
        # adjoint partner so that H stays Hermitian: conj(coef) (K^b A^T K^a) (x) R^T
        at = sp.csr_matrix(a.T)
        rpt, cit, vat = _csr_fields(at)
        rbt = np.stack([np.stack([_band_transpose(rb[sp_, s_], nr, hb) for sp_ in range(2)]) for s_ in range(2)])
        terms.append(CouplingTerm(rpt, cit, vat, rbt, (kp[1], kp[0]), coef.conjugate(), m % 2))
    op = OperatorDesc(nr=nr, nang=nang, hb=hb, kappa=kappa, h_poly=h_poly, s_poly=s_poly, terms=terms,
                      n_fields=2, h_chan=h_chan)
    psi0 = _random_state(rng, 1, nang, nr)
    pulses = [[Pulse(0.8, 50.0, 0.9, 0.3, True), Pulse(0.5, 1e9, 0.4, 1.0, False)]]
    return Workload("tiny", op, psi0, pulses, dt=0.05, t0=3.0, n_steps=np.array([4], dtype=np.int32),
                    tol=1e-12, meta={"seed": seed})


def _band_transpose(band, nr, hb):
    """Band of R^T from the band of R: R^T[i][i+d] = R[i+d][i] = band[-d+hb][i+d]."""
    out = np.zeros_like(band)
    idx = np.arange(nr)
    for d in range(-hb, hb + 1):
        ok = (idx + d >= 0) & (idx + d < nr)
        out[d + hb][ok] = band[-d + hb][idx[ok] + d]
    return out


band_transpose = _band_transpose
