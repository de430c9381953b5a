"""T_c(Dcut) by bisection on the oracle's X^(n) (Sec. 3, Eqs. (3.2)-(3.3)).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product path.

The paper runs the pure-tensor flow until X^(n) = (Tr A)^2 / Tr A^2 settles
(X -> 1 disordered, X -> 2 ordered, the Z2-broken fixed point having two equal
largest singular values of A) and reports T_c(Dcut) as lying between the
temperatures whose settled X differ.  This module does that with the oracle's
own flows: every point is a fresh oracle run at h = 0 (impurities off), the
phase is X > 3/2, and the bracket is halved each round.

Pinned by tests/test_oracle_pins.py: in d = 2 the bracket found at Dcut = 8
lies within 5e-4 (relative) of Onsager's beta_c = ln(1 + sqrt 2) / 2, and X
takes its two limits deep in either phase.
"""
from __future__ import annotations

from . import hotrg as H


def final_x(beta: float, dcut: int, d: int, nsteps: int) -> float:
    """X^(n) after nsteps steps (axes cycling 0..d-1) of a pure-T flow at h = 0."""
    f = H.run(beta, 0.0, dcut, d=d, nsteps=nsteps, impurities=False)
    return f.records[-1].X


def bisect(dcut: int, d: int, beta_lo: float, beta_hi: float, iterations: int, nsteps: int) -> dict:
    """Halve [beta_lo, beta_hi] `iterations` times, keeping the disordered end
    low and the ordered end high.  Returns the bracket and each (beta, X)."""
    points = []
    x_lo = final_x(beta_lo, dcut, d, nsteps)
    x_hi = final_x(beta_hi, dcut, d, nsteps)
    points += [(beta_lo, x_lo), (beta_hi, x_hi)]
    if not (x_lo < 1.5 < x_hi):
        raise ValueError(f"no transition inside [{beta_lo}, {beta_hi}]: X = {x_lo}, {x_hi}")
    lo, hi = beta_lo, beta_hi
    for _ in range(iterations):
        mid = (lo + hi) / 2
        x = final_x(mid, dcut, d, nsteps)
        points.append((mid, x))
        if x > 1.5:
            hi = mid
        else:
            lo = mid
    return {"beta_lo": lo, "beta_hi": hi, "points": points}
