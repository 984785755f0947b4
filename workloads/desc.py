"""Operator and workload descriptions shared by the GPU library and the oracle.

This module only holds data containers and (de)serialisation. It performs none of
the time-step arithmetic (no apply, no solve, no field evaluation); the GPU path and
the oracle each implement those on their own.

Operator (paper Sec. 2.2, eq. fullH): the state is stored channel-major as
``x[b][j][s][i]`` (instance, angular channel, spinor component P/Q, radial index).
The Hamiltonian acting on it is

    H(t) = H0 + sum_m coef_m * f_{field_m}(t) * (K^a A_m K^b) (x) R_m

where
  * H0 is block diagonal over channels j; block j couples (s, i) with (s', i+d)
    through ``sum_n kappa_j^n h_poly[n][s][s'][d+hb][i]`` (the kappa polynomial of
    eq. fullH) plus an optional per-channel complex band ``h_chan[j][s][s'][d+hb][i]``.
  * S (overlap) is the identity when ``s_poly`` has zero terms, else
    ``sum_n kappa_j^n s_poly[n]`` in the same band format.
  * each coupling term m has a real sparse angular matrix A_m (CSR over channels),
    exponents (a, b) so that the effective angular entry is
    ``kappa_j^a * A_m[j][j'] * kappa_j'^b``, a real radial 2x2-banded matrix
    ``r_band[s][s'][d+hb][i]``, a complex prefactor coef_m and a field index.

Band convention: ``band[s][s'][d+hb][i]`` multiplies ``x[s'][i+d]`` into ``y[s][i]``;
entries whose column i+d falls outside [0, nr) are zero.
"""
from __future__ import annotations

import dataclasses
import json
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

C_LIGHT = 137.036  # speed of light in atomic units used by the workloads


@dataclass
class CouplingTerm:
    a_rowptr: np.ndarray  # int32 [nang+1]
    a_col: np.ndarray  # int32 [nnz]
    a_val: np.ndarray  # float64 [nnz]
    r_band: np.ndarray  # float64 [2][2][2hb+1][nr]
    kpow: tuple  # (a, b): row-channel and column-channel kappa exponents
    coef: complex  # fixed complex prefactor
    field: int  # index of the time function multiplying this term


@dataclass
class OperatorDesc:
    nr: int
    nang: int
    hb: int
    kappa: np.ndarray  # float64 [nang]
    h_poly: np.ndarray  # float64 [n_h][2][2][2hb+1][nr]
    s_poly: np.ndarray  # float64 [n_s][2][2][2hb+1][nr]; n_s == 0 -> S = I
    terms: List[CouplingTerm]
    n_fields: int
    h_chan: Optional[np.ndarray] = None  # complex128 [nang][2][2][2hb+1][nr]

    @property
    def n_unknowns(self) -> int:
        return self.nang * 2 * self.nr


@dataclass
class Pulse:
    """Parameters of one time function f(t) = amp * env(t) * sin(omega t + phase).

    env(t) = sin^2(pi t / T) when ``envelope`` is true, else 1; f vanishes outside
    0 < t < T (finite-duration pulse of eq. ndpPot, dipole limit).
    """

    amp: float
    T: float
    omega: float
    phase: float
    envelope: bool = True


@dataclass
class Workload:
    name: str
    op: OperatorDesc
    psi0: np.ndarray  # complex128 [batch][nang][2][nr]
    pulses: list  # [batch][n_fields] of Pulse
    dt: float
    t0: float
    n_steps: np.ndarray  # int32 [batch]
    tol: float = 1e-12
    meta: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return self.psi0.shape[0]


def pulses_to_array(pulses) -> np.ndarray:
    """[batch][n_fields] Pulse -> float64 [batch][n_fields][5] (amp, T, omega, phase, envelope)."""
    out = np.zeros((len(pulses), len(pulses[0]), 5))
    for b, row in enumerate(pulses):
        for m, p in enumerate(row):
            out[b, m] = (p.amp, p.T, p.omega, p.phase, 1.0 if p.envelope else 0.0)
    return out


def pulses_from_array(arr) -> list:
    return [[Pulse(float(p[0]), float(p[1]), float(p[2]), float(p[3]), bool(p[4] != 0)) for p in row] for row in arr]


def save_workload(w: Workload, path: str) -> None:
    op = w.op
    arrays = {
        "kappa": op.kappa,
        "h_poly": op.h_poly,
        "s_poly": op.s_poly,
        "psi0": w.psi0,
        "pulses": pulses_to_array(w.pulses),
        "n_steps": w.n_steps,
    }
    if op.h_chan is not None:
        arrays["h_chan"] = op.h_chan
    for m, t in enumerate(op.terms):
        arrays[f"t{m}_rowptr"] = t.a_rowptr
        arrays[f"t{m}_col"] = t.a_col
        arrays[f"t{m}_val"] = t.a_val
        arrays[f"t{m}_r"] = t.r_band
    header = {
        "name": w.name, "nr": op.nr, "nang": op.nang, "hb": op.hb, "n_fields": op.n_fields,
        "dt": w.dt, "t0": w.t0, "tol": w.tol, "meta": w.meta,
        "terms": [{"kpow": list(t.kpow), "coef": [t.coef.real, t.coef.imag], "field": t.field} for t in op.terms],
    }
    arrays["header"] = np.frombuffer(json.dumps(header).encode(), dtype=np.uint8)
    np.savez(path, **arrays)


def load_workload(path: str) -> Workload:
    z = np.load(path, allow_pickle=False)
    h = json.loads(bytes(z["header"]).decode())
    terms = []
    for m, t in enumerate(h["terms"]):
        terms.append(CouplingTerm(z[f"t{m}_rowptr"], z[f"t{m}_col"], z[f"t{m}_val"], z[f"t{m}_r"],
                                  tuple(t["kpow"]), complex(*t["coef"]), int(t["field"])))
    op = OperatorDesc(h["nr"], h["nang"], h["hb"], z["kappa"], z["h_poly"], z["s_poly"], terms,
                      h["n_fields"], z["h_chan"] if "h_chan" in z.files else None)
    return Workload(h["name"], op, z["psi0"], pulses_from_array(z["pulses"]), h["dt"], h["t0"],
                    z["n_steps"], h["tol"], h["meta"])


def replace(w: Workload, **kw) -> Workload:
    return dataclasses.replace(w, **kw)
