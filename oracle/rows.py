"""Element-wise definition of y = a_S S x + a_H H(t) x at selected output rows (oracle).

Each output entry y[j][s][i] is written straight from eq. fullH without assembling a
matrix:

  (H0 x)[j][s][i]  = sum_{s', d} (sum_n kappa_j^n h_n[s][s'][d][i] + h_chan[j][s][s'][d][i]) x[j][s'][i+d]
  (V_m x)[j][s][i] = sum_{j'} kappa_j^a A_m[j][j'] kappa_j'^b sum_{s', d} R_m[s][s'][d][i] x[j'][s'][i+d]

It serves two purposes: a brute-force check of the CSR assembly on tiny inputs, and
sampled parity at sizes whose CSR matrix does not fit in memory.
"""
from __future__ import annotations

import numpy as np


def apply_rows(op, fvals, a_s: complex, a_h: complex, x: np.ndarray, rows) -> np.ndarray:
    """x: complex [nang][2][nr]; rows: flat indices j*2nr + s*nr + i. Returns y at those rows."""
    nr, hb = op.nr, op.hb
    out = np.zeros(len(rows), dtype=np.complex128)
    for k, row in enumerate(rows):
        j, rem = divmod(int(row), 2 * nr)
        s, i = divmod(rem, nr)
        kap = float(op.kappa[j])
        hx = 0.0 + 0.0j
        sx = 0.0 + 0.0j
        for s2 in range(2):
            for d in range(-hb, hb + 1):
                c = i + d
                if c < 0 or c >= nr:
                    continue
                tap = 0.0 + 0.0j
                for n in range(op.h_poly.shape[0]):
                    tap += kap ** n * op.h_poly[n, s, s2, d + hb, i]
                if op.h_chan is not None:
                    tap += op.h_chan[j, s, s2, d + hb, i]
                hx += tap * x[j, s2, c]
                if op.s_poly.shape[0] > 0:
                    stap = sum(kap ** n * op.s_poly[n, s, s2, d + hb, i] for n in range(op.s_poly.shape[0]))
                    sx += stap * x[j, s2, c]
        if op.s_poly.shape[0] == 0:
            sx = x[j, s, i]
        for t in op.terms:
            scale = t.coef * fvals[t.field]
            if scale == 0:
                continue
            acc = 0.0 + 0.0j
            for p in range(t.a_rowptr[j], t.a_rowptr[j + 1]):
                jj = int(t.a_col[p])
                w = kap ** t.kpow[0] * t.a_val[p] * float(op.kappa[jj]) ** t.kpow[1]
                for s2 in range(2):
                    for d in range(-hb, hb + 1):
                        c = i + d
                        if 0 <= c < nr:
                            acc += w * t.r_band[s, s2, d + hb, i] * x[jj, s2, c]
            hx += scale * acc
        out[k] = a_s * sx + a_h * hx
    return out
