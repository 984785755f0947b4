"""CSR assembly of the Hamiltonian and overlap (oracle).

Restates paper eq. fullH in the storage order x[j][s][i] (channel, spinor component,
radial index), flat index j*(2*nr) + s*nr + i:

  H0 = blockdiag_j( sum_n kappa_j^n h_n  [+ per-channel complex block] )     (kappa polynomial)
  S  = blockdiag_j( sum_n kappa_j^n s_n )  or I                            (overlap, Sec. 2.3)
  V_m = (K^a A_m K^b) kron R_m,  K = diag(kappa)                           (Kronecker coupling)
  H(t) = H0 + sum_m coef_m f_{field_m}(t) V_m

R_m, h_n, s_n are 2x2 grids of banded nr x nr blocks (Sec. 2.2: diagonal band plus
the P-Q bands). Assembly uses scipy.sparse kron / block_diag as library primitives.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def band_block(band: np.ndarray, nr: int, hb: int) -> sp.csr_matrix:
    """band[d+hb][i] (entry (i, i+d)) -> sparse nr x nr matrix."""
    rows, cols, vals = [], [], []
    idx = np.arange(nr)
    for d in range(-hb, hb + 1):
        ok = (idx + d >= 0) & (idx + d < nr)
        rows.append(idx[ok]); cols.append(idx[ok] + d); vals.append(band[d + hb][ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nr, nr))


def radial_2x2(bands: np.ndarray, nr: int, hb: int) -> sp.csr_matrix:
    """bands[s][s'][d+hb][i] -> the 2nr x 2nr radial matrix [[B00, B01], [B10, B11]]."""
    return sp.bmat([[band_block(bands[s][s2], nr, hb) for s2 in range(2)] for s in range(2)], format="csr")


def kappa_poly_block(poly: np.ndarray, kappa: float, nr: int, hb: int) -> sp.csr_matrix:
    """sum_n kappa^n poly[n] as a 2nr x 2nr matrix (eq. fullH, last line)."""
    m = sp.csr_matrix((2 * nr, 2 * nr), dtype=np.float64)
    for n in range(poly.shape[0]):
        m = m + (kappa ** n) * radial_2x2(poly[n], nr, hb)
    return m


def h0_csr(op) -> sp.csr_matrix:
    blocks = []
    for j in range(op.nang):
        b = kappa_poly_block(op.h_poly, float(op.kappa[j]), op.nr, op.hb).astype(np.complex128)
        if op.h_chan is not None:
            b = b + radial_2x2(op.h_chan[j], op.nr, op.hb)
        blocks.append(b)
    return sp.block_diag(blocks, format="csr")


def s_csr(op) -> sp.csr_matrix:
    n = op.nang * 2 * op.nr
    if op.s_poly.shape[0] == 0:
        return sp.identity(n, dtype=np.complex128, format="csr")
    blocks = [kappa_poly_block(op.s_poly, float(op.kappa[j]), op.nr, op.hb) for j in range(op.nang)]
    return sp.block_diag(blocks, format="csr").astype(np.complex128)


def term_csr(op, term) -> sp.csr_matrix:
    """V_m = (K^a A_m K^b) kron R_m."""
    a = sp.csr_matrix((term.a_val, term.a_col, term.a_rowptr), shape=(op.nang, op.nang))
    ka = sp.diags(op.kappa ** term.kpow[0])
    kb = sp.diags(op.kappa ** term.kpow[1])
    ang = ka @ a @ kb
    return sp.kron(ang, radial_2x2(term.r_band, op.nr, op.hb), format="csr")


class Assembled:
    """H0, S and the coupling matrices of one operator, assembled once (Sec. 2.2: H0 and the
    radial integrals are computed once; H(t) is recombined every step)."""

    def __init__(self, op):
        self.op = op
        self.H0 = h0_csr(op)
        self.S = s_csr(op)
        self.V = [term_csr(op, t) for t in op.terms]

    def hamiltonian(self, fvals) -> sp.csr_matrix:
        H = self.H0.copy()
        for t, v in zip(self.op.terms, self.V):
            H = H + (t.coef * fvals[t.field]) * v
        return H.tocsr()

    def operator(self, fvals, a_s: complex, a_h: complex) -> sp.csr_matrix:
        """a_S S + a_H H(t)."""
        return (a_s * self.S + a_h * self.hamiltonian(fvals)).tocsr()


def channel_rows(op, fvals, a_s: complex, a_h: complex, j0: int, j1: int) -> sp.csr_matrix:
    """Rows of channels [j0, j1) of a_S S + a_H H(t): the same construction as the full assembly
    (eq. fullH), restricted to those block rows, as a ((j1-j0) 2nr) x (nang 2nr) CSR matrix. Used
    where the whole matrix does not fit in memory (sampled parity, timing of a row slice)."""
    nr, hb, nang = op.nr, op.hb, op.nang
    n = 2 * nr
    blocks = []
    for j in range(j0, j1):
        b = kappa_poly_block(op.h_poly, float(op.kappa[j]), nr, hb).astype(np.complex128)
        if op.h_chan is not None:
            b = b + radial_2x2(op.h_chan[j], nr, hb)
        if op.s_poly.shape[0] == 0:
            sb = sp.identity(n, dtype=np.complex128, format="csr")
        else:
            sb = kappa_poly_block(op.s_poly, float(op.kappa[j]), nr, hb).astype(np.complex128)
        blocks.append(a_s * sb + a_h * b)
    diag = sp.block_diag(blocks, format="csr")
    left = sp.csr_matrix(((j1 - j0) * n, j0 * n), dtype=np.complex128)
    right = sp.csr_matrix(((j1 - j0) * n, (nang - j1) * n), dtype=np.complex128)
    out = sp.hstack([left, diag, right], format="csr")
    for t in op.terms:
        scale = a_h * t.coef * fvals[t.field]
        if scale == 0:
            continue
        a = sp.csr_matrix((t.a_val, t.a_col, t.a_rowptr), shape=(nang, nang))
        ang = (sp.diags(op.kappa ** t.kpow[0]) @ a @ sp.diags(op.kappa ** t.kpow[1])).tocsr()[j0:j1]
        out = out + scale * sp.kron(ang, radial_2x2(t.r_band, nr, hb), format="csr")
    return out.tocsr()
