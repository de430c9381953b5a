"""Energy and magnetisation jumps at T_c(Dcut) from oracle flows (Sec. 3).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product path.

The paper reads the internal energy from the impure-tensor method at h = 0
and the magnetisation <sigma> at h = 1e-9 and 2e-9, taken to h -> 0 along a
straight line; at T_c each has a finite jump, found by straight-line
extrapolation toward T_c from the low- and the high-temperature side.  Here
every number comes from `oracle.hotrg.run` (impurities on); the lines are
ordinary least squares (numpy.polyfit of degree one).

Pinned by tests/test_oracle_pins.py: in d = 2 the zero-field limit of m at
Dcut = 8 equals Onsager's spontaneous magnetisation within 1e-4 (beta = 0.5)
and 1e-6 (beta = 0.6), and vanishes in the disordered phase; the straight-line
step is a library routine.
"""
from __future__ import annotations

import numpy as np

from . import hotrg as H


def last_step(beta: float, h: float, dcut: int, d: int, nsteps: int):
    """StepRecord of the last step of a flow with impurities."""
    return H.run(beta, h, dcut, d=d, nsteps=nsteps, impurities=True).records[-1]


def spontaneous_m(beta: float, dcut: int, d: int, nsteps: int, h1: float = 1e-9, h2: float = 2e-9):
    """(m at h -> 0, m(h1), m(h2)): m is linear in h between the two fields."""
    m1 = last_step(beta, h1, dcut, d, nsteps).m_imp
    m2 = last_step(beta, h2, dcut, d, nsteps).m_imp
    slope = (m2 - m1) / (h2 - h1)
    return m1 - slope * h1, m1, m2


def jumps(dcut: int, d: int, t_c: float, temps, nsteps: int, h1: float = 1e-9, h2: float = 2e-9) -> dict:
    """Per temperature: e at h = 0 and m at h -> 0; then the jumps at t_c."""
    rows = []
    for T in sorted(temps):
        beta = 1.0 / T
        e = last_step(beta, 0.0, dcut, d, nsteps).e_imp
        m0, m1, m2 = spontaneous_m(beta, dcut, d, nsteps, h1, h2)
        rows.append((T, e, m0, m1, m2))
    lo = [r for r in rows if r[0] < t_c]
    hi = [r for r in rows if r[0] > t_c]

    def at_tc(side, col):
        a, b = np.polyfit([r[0] for r in side], [r[col] for r in side], 1)
        return a * t_c + b

    return {"rows": rows,
            "delta_e": at_tc(hi, 1) - at_tc(lo, 1),
            "delta_m": at_tc(lo, 2) - at_tc(hi, 2)}
