"""First-order jumps of the energy and the magnetisation at T_c(Dcut) (Sec. 3).

Energy: the impurity estimator of Eqs. (2.7) and (2.10) at h = 0, per site
e = -4 <sigma_i sigma_j> (the pair along the first coarse-graining axis).
Magnetisation: the one-impurity estimator of Eqs. (2.11)-(2.12) at two small
fields h1 and h2 (the paper takes 1e-9 and 2e-9), continued linearly to
h -> 0.  Both are read at the flow's last step (the largest lattice).  For
each observable a least-squares straight line in T through the points below
T_c and one through the points above are evaluated at T_c; the jump is their
difference (Delta E = E(T_c+) - E(T_c-), Delta m = m(T_c-) - m(T_c+)).
Every flow runs on the GPU through the HIP library; this module is host
bookkeeping.
"""
from __future__ import annotations

from . import hotrg as H


def final_observables(beta: float, h: float, dcut: int, nsteps: int = 40, precision: int = H.FP64,
                      **ctx_kw) -> dict:
    """Observables after nsteps steps of a flow with both impurity tensors."""
    with H.Context(beta, h, dcut, precision=precision, impurities=True, **ctx_kw) as ctx:
        for n in range(nsteps):
            ctx.step(n % 4)
        return ctx.observables()


def zero_field_limit(y1: float, y2: float, h1: float, h2: float) -> float:
    """Value at h = 0 of the straight line through (h1, y1) and (h2, y2)."""
    if h1 == h2:
        raise ValueError("need two distinct fields")
    return (h2 * y1 - h1 * y2) / (h2 - h1)


def line_value(ts, ys, t0: float) -> float:
    """Least-squares straight line through (ts, ys), evaluated at t0."""
    n = len(ts)
    if n != len(ys) or n < 2:
        raise ValueError("need at least two points per side")
    tm = sum(ts) / n
    ym = sum(ys) / n
    stt = sum((t - tm) ** 2 for t in ts)
    if stt == 0.0:
        raise ValueError("points of one side share one temperature")
    slope = sum((t - tm) * (y - ym) for t, y in zip(ts, ys)) / stt
    return ym + slope * (t0 - tm)


def point(beta: float, dcut: int, nsteps: int, h1: float, h2: float, precision: int, **ctx_kw) -> dict:
    """Energy at h = 0 and the zero-field magnetisation at one temperature."""
    o0 = final_observables(beta, 0.0, dcut, nsteps, precision, **ctx_kw)
    o1 = final_observables(beta, h1, dcut, nsteps, precision, **ctx_kw)
    o2 = final_observables(beta, h2, dcut, nsteps, precision, **ctx_kw)
    return {"beta": beta, "T": 1.0 / beta, "e": o0["e_imp"], "X": o0["X"],
            "m_h1": o1["m_imp"], "m_h2": o2["m_imp"],
            "m": zero_field_limit(o1["m_imp"], o2["m_imp"], h1, h2)}


def jumps_from_points(points, t_c: float) -> dict:
    """Delta E and Delta m from per-temperature points on both sides of t_c."""
    low = [p for p in points if p["T"] < t_c]
    high = [p for p in points if p["T"] > t_c]
    e_low = line_value([p["T"] for p in low], [p["e"] for p in low], t_c)
    e_high = line_value([p["T"] for p in high], [p["e"] for p in high], t_c)
    m_low = line_value([p["T"] for p in low], [p["m"] for p in low], t_c)
    m_high = line_value([p["T"] for p in high], [p["m"] for p in high], t_c)
    return {"T_c": t_c, "e_below": e_low, "e_above": e_high, "delta_e": e_high - e_low,
            "m_below": m_low, "m_above": m_high, "delta_m": m_low - m_high}


def first_order_jumps(dcut: int, t_c: float, temps, nsteps: int = 40, h1: float = 1e-9, h2: float = 2e-9,
                      precision: int = H.FP64, **ctx_kw) -> dict:
    """Evaluate every temperature in `temps` (some below t_c, some above) and
    return the jumps and the points."""
    pts = [point(1.0 / T, dcut, nsteps, h1, h2, precision, **ctx_kw) for T in sorted(temps)]
    out = jumps_from_points(pts, t_c)
    out.update(points=pts, dcut=dcut, nsteps=nsteps, h1=h1, h2=h2)
    return out
