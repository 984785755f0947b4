"""Pins of the oracle's pulse and of BiCGSTAB's restart and breakdown branches (no GPU).

The pulse of eq. ndpPot (dipole limit) is checked against facts that do not restate its
formula: the product-to-sum factorisation into three carriers that eq. bdpA's time functions
rest on, evaluated term by term through complex exponentials; a closed-form time integral over
the whole pulse; hand-computed points. Planted mistakes (a sin envelope instead of sin^2, a
cosine carrier, a doubled envelope frequency) must fail these pins.

BiCGSTAB (van der Vorst 1992) is driven through its three restart paths on small systems whose
arithmetic is exact in binary floating point (small integers and dyadic fractions), so the
vanishing scalars are exactly zero: a shadow residual orthogonal to r0 (rho = 0), one
orthogonal to A r0 (<r^, v> = 0), and a tolerance below what FP64 attains (the true-residual
check fails and the solve restarts from its iterate). Each must still agree with LAPACK.
"""
import cmath
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import fields
from oracle.bicgstab import bicgstab
from workloads.desc import Pulse


# ---------------------------------------------------------------- pulse (eq. ndpPot, eq. bdpA)

def _three_carriers(amp, T, w, phi, t):
    """sin^2(pi t/T) sin(w t + phi) = 1/2 sin(w t + phi) - 1/4 sin((w + W) t + phi) - 1/4 sin((w - W) t + phi),
    W = 2 pi / T, each carrier taken as the imaginary part of a complex exponential."""
    W = 2 * math.pi / T
    c0 = cmath.exp(1j * (w * t + phi)).imag
    cp = cmath.exp(1j * ((w + W) * t + phi)).imag
    cm = cmath.exp(1j * ((w - W) * t + phi)).imag
    return amp * (0.5 * c0 - 0.25 * cp - 0.25 * cm)


def _pulse_integral(amp, T, w, phi):
    """Closed form of the integral of the pulse over (0, T): the three carriers integrated,
    int_0^T sin(a t + phi) dt = (cos(phi) - cos(a T + phi)) / a."""
    W = 2 * math.pi / T

    def carrier(a):
        return (math.cos(phi) - math.cos(a * T + phi)) / a
    return amp * (0.5 * carrier(w) - 0.25 * carrier(w + W) - 0.25 * carrier(w - W))


PULSES = [Pulse(0.05, 20.0, 0.057, math.pi / 2, True), Pulse(1.7, 881.85, 0.057, 0.3, True),
          Pulse(0.4, 6.0, 62.83, 2.1, True)]


def _check_pulse(fn, p):
    rng = np.random.default_rng(11)
    ts = rng.uniform(0.0, p.T, 200)
    err = max(abs(fn(p, t) - _three_carriers(p.amp, p.T, p.omega, p.phase, t)) for t in ts)
    integ, _ = integrate.quad(lambda t: fn(p, t), 0.0, p.T, limit=2000, epsabs=1e-13, epsrel=1e-11)
    ref = _pulse_integral(p.amp, p.T, p.omega, p.phase)
    return err, abs(integ - ref)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("k", range(len(PULSES)))
def test_pulse_matches_three_carrier_factorisation_and_integral(k):
    """eq. bdpA: the sin^2 pulse is a sum of three sine carriers at w and w +- 2 pi/T."""
    p = PULSES[k]
    err, ierr = _check_pulse(fields.pulse_value, p)
    assert err < 1e-14 * max(1.0, p.amp)
    assert ierr < 1e-9 * max(1.0, p.amp)


def test_pulse_hand_points():
    """Hand-computed points: the envelope peak at t = T/2 and the carrier phase."""
    p = Pulse(2.0, 10.0, math.pi / 10, 0.0, True)  # omega T / 2 = pi / 2
    assert abs(fields.pulse_value(p, 5.0) - 2.0) < 1e-15
    q = Pulse(2.0, 10.0, math.pi / 10, math.pi / 2, True)  # cosine carrier: cos(pi/2) = 0 at the peak
    assert abs(fields.pulse_value(q, 5.0)) < 1e-15
    r = Pulse(3.0, 8.0, 0.0, math.pi / 2, True)  # no carrier: the bare envelope, sin^2(pi/4) = 1/2 at t = 2
    assert abs(fields.pulse_value(r, 2.0) - 1.5) < 1e-15
    assert fields.pulse_value(p, 0.0) == 0.0 and fields.pulse_value(p, 10.0) == 0.0


def _planted_sin_envelope(p, t):
    if not (0.0 < t < p.T):
        return 0.0
    return p.amp * math.sin(math.pi * t / p.T) * math.sin(p.omega * t + p.phase)


def _planted_cos_carrier(p, t):
    if not (0.0 < t < p.T):
        return 0.0
    return p.amp * math.sin(math.pi * t / p.T) ** 2 * math.cos(p.omega * t + p.phase)


def _planted_double_freq(p, t):
    if not (0.0 < t < p.T):
        return 0.0
    return p.amp * math.sin(2 * math.pi * t / p.T) ** 2 * math.sin(p.omega * t + p.phase)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("planted", [_planted_sin_envelope, _planted_cos_carrier, _planted_double_freq])
def test_planted_pulse_mistakes_are_caught(planted):
    for p in PULSES:
        err, ierr = _check_pulse(planted, p)
        assert err > 1e-3 * p.amp


# ---------------------------------------------------------------- BiCGSTAB branches

A3 = np.array([[2, 1, 0], [0, 3, 1], [1, 0, 4]], dtype=np.complex128)
B3 = np.array([1, 2, 3], dtype=np.complex128)


def test_rho_breakdown_restarts_and_converges():
    """Shadow residual orthogonal to r0: rho = <r^, r0> = 0 exactly; the restart takes r^ = r."""
    rhat = np.array([2, -1, 0], dtype=np.complex128)
    assert np.vdot(rhat, B3) == 0
    x, st = bicgstab(A3, B3, None, tol=1e-13, rhat0=rhat)
    assert st.restarts >= 1 and st.converged
    assert np.linalg.norm(x - np.linalg.solve(A3, B3)) <= 1e-12 * np.linalg.norm(x)


def test_rv_breakdown_restarts_and_converges():
    """Shadow residual orthogonal to v = A p (p = r0 in the first iteration): <r^, v> = 0 exactly
    while rho != 0; the iteration cannot form alpha and restarts."""
    rhat = np.array([9, -4, 0], dtype=np.complex128)
    assert np.vdot(rhat, A3 @ B3) == 0 and np.vdot(rhat, B3) != 0
    x, st = bicgstab(A3, B3, None, tol=1e-13, rhat0=rhat)
    assert st.restarts >= 1 and st.converged
    assert np.linalg.norm(x - np.linalg.solve(A3, B3)) <= 1e-12 * np.linalg.norm(x)


def test_unattainable_tolerance_restarts_from_true_residual():
    """A tolerance below what FP64 attains: the recursive residual passes, the true residual check
    fails, and the solve restarts from its iterate until max_iter; the iterate stays the LAPACK one."""
    rng = np.random.default_rng(5)
    n = 12
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * 0.3
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, st = bicgstab(A, b, None, tol=1e-30, max_iter=60)
    assert not st.converged and st.restarts >= 1
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)


def test_repeated_breakdown_terminates():
    """A Krylov space that breaks down again after every restart: omega = 0 exactly in the first
    iteration (t = A s orthogonal to s), then <r^, v> = 0 in every restarted cycle. The solve must
    end unconverged after the restart bound instead of looping."""
    K = np.array([[0, 1, 1, 2], [-1, 0, 1, 1], [-1, -1, 0, 1], [-2, -1, -1, 0]], dtype=np.complex128)
    A = K + np.diag([4, 0, 0, 0]).astype(np.complex128)
    b = np.ones(4, dtype=np.complex128)
    rhat = np.array([1, 0, 0, 0], dtype=np.complex128)
    x, st = bicgstab(A, b, None, tol=1e-12, max_iter=100, rhat0=rhat, max_restarts=5)
    assert not st.converged and st.restarts > 5
    assert np.all(np.isfinite(x))
