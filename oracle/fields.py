"""Laser time functions (oracle).

Dipole limit of the sin^2-envelope pulse of paper eq. ndpPot: the vector potential
amplitude is amp * sin^2(pi t / T) * sin(omega t + phase) for 0 < t < T and zero
otherwise. The beyond-dipole form (eq. bdpA) factorises the pulse into a sum of such
time functions f_alpha(t) (sines and cosines at omega and omega +- 2 pi / T); a cosine
is a sine with phase pi/2. ``envelope = False`` drops the sin^2 factor.
"""
from __future__ import annotations

import math


def pulse_value(p, t: float) -> float:
    """f(t) for one pulse (attributes amp, T, omega, phase, envelope)."""
    if not (0.0 < t < p.T):
        return 0.0
    env = math.sin(math.pi * t / p.T) ** 2 if p.envelope else 1.0
    return p.amp * env * math.sin(p.omega * t + p.phase)


def field_values(pulses_row, t: float):
    """[n_fields] values of every time function of one instance at time t."""
    return [pulse_value(p, t) for p in pulses_row]


def midpoint_time(t_n: float, dt: float) -> float:
    """The Hamiltonian of one step is taken at t_n + dt/2 (midpoint rule, Sec. 2.4)."""
    return t_n + 0.5 * dt
