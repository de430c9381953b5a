"""Transition temperature at fixed Dcut from the X indicator (Sec. 3, Eqs. (3.2)-(3.3)).

After a step along axis mu, A^(n) is the Dcut x Dcut matrix left when every
axis but mu has its two legs traced (Eq. (3.2)), and X^(n) = (Tr A)^2 / Tr A^2
(Eq. (3.3)) counts how many singular values of A share the largest one.  A
disordered-phase flow ends at a tensor with one dominant value (X -> 1); an
ordered-phase flow ends at the Z2-broken fixed point with two (X -> 2).  The
paper iterates until X^(n) settles (n beyond 30) and places T_c(Dcut) between
temperatures whose converged X differ.  Here that bracket is narrowed by
bisection in beta; every X comes from a pure-T flow at h = 0 run by the HIP
library (hotrg_step, then hotrg_observables, which evaluates Eqs. (3.2)-(3.3)
on the device).  The bisection itself is host bookkeeping.
"""
from __future__ import annotations

import math

from . import hotrg as H

X_THRESHOLD = 1.5    # halfway between the disordered (1) and ordered (2) limits
CONVERGED_TOL = 0.05


def x_history(beta: float, dcut: int, nsteps: int = 40, precision: int = H.FP64, **ctx_kw) -> list:
    """X^(n) after every step of a pure-T flow at h = 0, axes cycling x, y, z, t."""
    xs = []
    with H.Context(beta, 0.0, dcut, precision=precision, impurities=False, **ctx_kw) as ctx:
        for n in range(nsteps):
            ctx.step(n % 4)
            xs.append(ctx.observables()["X"])
    return xs


def phase(x: float) -> int:
    """1 for the ordered phase (X near 2), 0 for the disordered phase (X near 1)."""
    if not math.isfinite(x):
        raise ValueError(f"X = {x} is not finite")
    return 1 if x > X_THRESHOLD else 0


def settled(x: float) -> bool:
    """True when X is within CONVERGED_TOL of one of the two limits."""
    return abs(x - 1.0) <= CONVERGED_TOL or abs(x - 2.0) <= CONVERGED_TOL


def bisect_transition(x_of_beta, beta_lo: float, beta_hi: float, iterations: int) -> dict:
    """Bisection on the phase of X(beta) inside [beta_lo, beta_hi].

    x_of_beta maps beta to the final X of a flow.  beta_lo must be in the
    disordered phase and beta_hi in the ordered phase (T_c lies between).
    Returns the final bracket and every evaluated point in evaluation order.
    """
    if not beta_lo < beta_hi:
        raise ValueError("need beta_lo < beta_hi")
    points = []

    def probe(beta):
        x = float(x_of_beta(beta))
        points.append({"beta": beta, "X": x, "phase": phase(x), "settled": settled(x)})
        return points[-1]["phase"]

    if probe(beta_lo) != 0:
        raise ValueError(f"beta_lo = {beta_lo} is not in the disordered phase (X = {points[-1]['X']})")
    if probe(beta_hi) != 1:
        raise ValueError(f"beta_hi = {beta_hi} is not in the ordered phase (X = {points[-1]['X']})")
    lo, hi = beta_lo, beta_hi
    for _ in range(iterations):
        mid = 0.5 * (lo + hi)
        if probe(mid):
            hi = mid
        else:
            lo = mid
    beta_c = 0.5 * (lo + hi)
    return {"beta_lo": lo, "beta_hi": hi, "beta_c": beta_c, "T_c": 1.0 / beta_c,
            "T_c_halfwidth": 0.5 * (1.0 / lo - 1.0 / hi), "points": points,
            "unsettled": sum(1 for p in points if not p["settled"])}


def bracket_by_scan(x_of_beta, betas) -> tuple:
    """First pair of neighbouring betas (ascending) whose phases differ, plus
    the scanned points; (None, points) when every point has the same phase."""
    betas = sorted(betas)
    points = []
    prev = None
    for b in betas:
        x = float(x_of_beta(b))
        points.append({"beta": b, "X": x, "phase": phase(x), "settled": settled(x)})
        if prev is not None and prev["phase"] == 0 and points[-1]["phase"] == 1:
            return (prev["beta"], b), points
        prev = points[-1]
    return None, points


def locate_tc(dcut: int, beta_lo: float, beta_hi: float, iterations: int = 10, nsteps: int = 40,
              precision: int = H.FP64, **ctx_kw) -> dict:
    """T_c(Dcut) bracket from the converged X of GPU flows (Sec. 3)."""
    res = bisect_transition(lambda b: x_history(b, dcut, nsteps, precision, **ctx_kw)[-1],
                            beta_lo, beta_hi, iterations)
    res.update(dcut=dcut, nsteps=nsteps)
    return res
