"""HOTRG for the d-dimensional Ising model, plain CPU float64 (test oracle).

TEST INFRASTRUCTURE ONLY: imported by tests/, smoke() and bench.py's
cpu_baseline leg, never by the product path.

Conventions (Sec. 2 of the paper, Eqs. (2.1)-(2.5)):
  * a site tensor has 2d legs; leg 2k is the backward leg of axis k, leg 2k+1
    the forward leg (x, x', y, y', z, z', t, t' in d = 4);
  * one coarse-graining step along axis mu merges a lower tensor T1 (site i)
    and an upper tensor T2 (site i + mu): T1's forward mu-leg is contracted
    with T2's backward mu-leg (the internal bond alpha of Eqs. (2.8)-(2.9));
  * every transverse axis nu != mu gets one isometry U_nu of shape
    (D_nu^2, k_nu), whose row index is i1 * D_nu + i2 with i1 a leg of T1 and
    i2 the same leg of T2.  The same U_nu is applied to the merged backward
    legs and to the merged forward legs (Eqs. (2.8)-(2.9));
  * the new tensor keeps T1's backward mu-leg and T2's forward mu-leg.

Readings of points the paper leaves open (each is listed with its reason in
the design notes):
  R1  U_nu comes from the eigen-decomposition of the environment of the
      merged backward legs or of the merged forward legs (HOSVD of the
      merged tensor M = T1 T2 along that leg), whichever discards less weight.
  R2  near-ties eps_b <= eps_f + 1e-11 * Tr E pick the backward side (both
      environments have the same trace, |M|^2).
  R3  a cut through a (near-)degenerate multiplet, gap
      (lam_k - lam_{k+1}) / lam_1 <= tau, drops back to the largest k' < Dcut
      whose gap exceeds tau.
  R4  when every bond carries a Z2 parity label and the environment has no
      entry between different parities, each parity block is diagonalised
      on its own (keeps the h = 0 symmetry exact).
  R5  per-step normalisation by the Frobenius norm c_n; the flow keeps
      lnZ/N = sum_k 2^-k ln c_k + 2^-n ln Tr T^(n).
  R6  the two-impurity pair of Eq. (2.7) lies along the first
      coarse-graining axis, so the first step is the S.S step of Eq. (2.8).
  R11 a merged leg with D_nu^2 <= Dcut is not truncated (U = identity).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TAU_DEGENERATE = 1e-12
SIDE_TIE = 1e-11


# ---------------------------------------------------------------------------
# Initial tensors: Sec. 2, Eq. (2.1) and the definitions of T^(0) (Eq. (2.2))
# and of the impure tensor S^(0) (Eq. (2.6)).
# ---------------------------------------------------------------------------
def bond_factor(beta: float) -> np.ndarray:
    """W = U sqrt(Lambda) for the bond matrix T_{ss'} = exp(beta s s').

    The bond matrix [[e^b, e^-b], [e^-b, e^b]] has eigenvectors
    (1, 1)/sqrt2 and (1, -1)/sqrt2 with eigenvalues 2 cosh b and 2 sinh b
    (Sec. 2, text after Eq. (2.1)).  Row 0 is sigma = +1, row 1 sigma = -1.
    Column 0 is Z2-even, column 1 Z2-odd.
    """
    if beta < 0:
        raise ValueError("beta must be >= 0 (ferromagnetic model)")
    c = math.sqrt(math.cosh(beta))
    s = math.sqrt(math.sinh(beta))
    return np.array([[c, s], [c, -s]], dtype=np.float64)


def site_tensors(beta: float, h: float, d: int) -> tuple[np.ndarray, np.ndarray]:
    """T^(0) and S^(0) of Eqs. (2.2) and (2.6), 2d legs of dimension 2.

    T^(0)_{i1..i2d} = sum_sigma V_sigma prod_k W[sigma, i_k],
    S^(0)           = the same sum with an extra factor sigma,
    V_sigma = exp(beta h sigma).
    """
    W = bond_factor(beta)
    T = np.zeros((2,) * (2 * d))
    S = np.zeros((2,) * (2 * d))
    for row, sigma in enumerate((1.0, -1.0)):
        outer = W[row]
        for _ in range(2 * d - 1):
            outer = np.multiply.outer(outer, W[row])
        v = math.exp(beta * h * sigma)
        T += v * outer
        S += sigma * v * outer
    return T, S


# ---------------------------------------------------------------------------
# Traces: Eq. (2.5), and the X^(n) indicator of Eqs. (3.2)-(3.3).
# ---------------------------------------------------------------------------
def trace(T: np.ndarray) -> float:
    """Tr T = sum T_{x x y y ...}: every backward leg joined to its forward leg."""
    out = T
    while out.ndim:
        out = np.trace(out, axis1=0, axis2=1)
    return float(out)


def a_matrix(T: np.ndarray, axis: int) -> np.ndarray:
    """A_{t t'} = sum over the diagonals of every other axis (Eq. (3.2))."""
    d = T.ndim // 2
    legs = list(range(2 * d))
    keep = [2 * axis, 2 * axis + 1]
    out = np.transpose(T, [l for l in legs if l not in keep] + keep)
    while out.ndim > 2:
        out = np.trace(out, axis1=0, axis2=1)
    return out


def x_indicator(T: np.ndarray, axis: int) -> float:
    """X = (Tr A)^2 / Tr(A^2) (Eq. (3.3))."""
    A = a_matrix(T, axis)
    return float(np.trace(A) ** 2 / np.trace(A @ A))


# ---------------------------------------------------------------------------
# Environments (HOSVD of the merged tensor, Sec. 2 and reading R1).
# ---------------------------------------------------------------------------
def _gram_pair(T: np.ndarray, leg: int, other: int) -> np.ndarray:
    """G[(p, a), (p~, a~)] = sum over all legs except {leg, other} of
    T[.. p .. a ..] T[.. p~ .. a~ ..]; returned with axes (p, a, p~, a~)."""
    rest = [l for l in range(T.ndim) if l not in (leg, other)]
    G = np.tensordot(T, T, axes=(rest, rest))
    # tensordot keeps the open legs in their original order
    if leg > other:
        G = G.transpose(1, 0, 3, 2)
    return G


def environment(T1: np.ndarray, T2: np.ndarray, mu: int, nu: int, side: int) -> np.ndarray:
    """E = M_(m) M_(m)^T for the merged leg m = (T1 leg, T2 leg) of axis nu.

    side 0 merges the backward legs, side 1 the forward legs.  M is the
    two-site tensor T1 .alpha T2 (alpha = T1's forward mu-leg = T2's backward
    mu-leg).  Summing M over every other leg factorises into two Grams:
        E[(p,q),(p~,q~)] = sum_{a,a~} G1[(p,a),(p~,a~)] G2[(q,a),(q~,a~)],
    G1 from T1 with open legs (nu side, mu forward), G2 from T2 with open
    legs (nu side, mu backward).
    """
    leg = 2 * nu + side
    G1 = _gram_pair(T1, leg, 2 * mu + 1)          # (p, a, p~, a~)
    G2 = _gram_pair(T2, leg, 2 * mu)              # (q, a, q~, a~)
    E = np.einsum("pauc,qavc->pquv", G1, G2, optimize=True)
    n1, n2 = T1.shape[leg], T2.shape[leg]
    return E.reshape(n1 * n2, n1 * n2)


def environment_direct(T1: np.ndarray, T2: np.ndarray, mu: int, nu: int, side: int) -> np.ndarray:
    """Same matrix built by materialising M (only for tiny tensors; a pin)."""
    d = T1.ndim // 2
    M = np.tensordot(T1, T2, axes=([2 * mu + 1], [2 * mu]))
    # M legs: T1 legs without 2mu+1 (2d-1 of them), then T2 legs without 2mu
    t1_legs = [l for l in range(2 * d) if l != 2 * mu + 1]
    t2_legs = [l for l in range(2 * d) if l != 2 * mu]
    leg = 2 * nu + side
    i1 = t1_legs.index(leg)
    i2 = len(t1_legs) + t2_legs.index(leg)
    rest = [i for i in range(M.ndim) if i not in (i1, i2)]
    Mm = np.transpose(M, [i1, i2] + rest).reshape(T1.shape[leg] * T2.shape[leg], -1)
    return Mm @ Mm.T


# ---------------------------------------------------------------------------
# Truncation: eigh, cut (R3), side choice (R1, R2), parity blocks (R4).
# ---------------------------------------------------------------------------
@dataclass
class Cut:
    k: int
    gap: float            # (lam_k - lam_{k+1}) / lam_1 at the chosen k (inf if untruncated)
    flagged: bool         # no k' < Dcut had a gap above tau


def choose_cut(lam: np.ndarray, dcut: int, tau: float = TAU_DEGENERATE) -> Cut:
    """Reading R3.  lam is sorted descending; returns how many to keep."""
    n = len(lam)
    if n <= dcut:
        return Cut(n, math.inf, False)
    lam1 = lam[0]
    if not lam1 > 0:
        return Cut(dcut, 0.0, True)
    gaps = (lam[:-1] - lam[1:]) / lam1        # gaps[k-1] = gap after the k-th value
    if gaps[dcut - 1] > tau:
        return Cut(dcut, float(gaps[dcut - 1]), False)
    for k in range(dcut - 1, 0, -1):
        if gaps[k - 1] > tau:
            return Cut(k, float(gaps[k - 1]), False)
    return Cut(dcut, float(gaps[dcut - 1]), True)


def merged_labels(l1, l2):
    if l1 is None or l2 is None:
        return None
    return (np.asarray(l1)[:, None] ^ np.asarray(l2)[None, :]).reshape(-1)


def eigh_desc(E: np.ndarray, labels=None):
    """Eigenpairs sorted by decreasing eigenvalue.

    With parity labels and an environment that has no entry between
    different parities (reading R4), each block is diagonalised separately
    and the eigenvectors inherit the block's label.  Returns (lam, V, lab)
    where lab is None when no labels are carried.
    """
    if labels is not None:
        lab = np.asarray(labels)
        off = lab[:, None] != lab[None, :]
        if not np.any(E[off] != 0.0):
            n = E.shape[0]
            lams, vecs, labs = [], [], []
            for p in (0, 1):
                idx = np.nonzero(lab == p)[0]
                if idx.size == 0:
                    continue
                w, v = np.linalg.eigh(E[np.ix_(idx, idx)])
                full = np.zeros((n, idx.size))
                full[idx, :] = v
                lams.append(w)
                vecs.append(full)
                labs.append(np.full(idx.size, p, dtype=np.int64))
            lam = np.concatenate(lams)
            V = np.concatenate(vecs, axis=1)
            lb = np.concatenate(labs)
            order = np.argsort(-lam, kind="stable")
            return lam[order], V[:, order], lb[order]
    w, v = np.linalg.eigh(E)
    order = np.argsort(-w, kind="stable")
    return w[order], v[:, order], None


@dataclass
class AxisDecision:
    nu: int
    side: int                      # 0 backward, 1 forward
    k: int
    eps: tuple                     # (eps_b, eps_f), discarded weight
    gap: float
    flagged: bool
    spectra: tuple                 # (lam_b, lam_f), descending
    truncated: bool


def isometries(T: np.ndarray, mu: int, dcut: int, labels=None, tau: float = TAU_DEGENERATE):
    """U_nu for every transverse axis nu of a step along mu (readings R1-R4, R11).

    Returns (Us, new_labels, decisions): Us[nu] is (D_nu^2, k_nu);
    new_labels[nu] the parity of each kept vector (or None).
    """
    d = T.ndim // 2
    Us, new_labels, decisions = {}, {}, []
    for nu in range(d):
        if nu == mu:
            continue
        D = T.shape[2 * nu]
        lab = merged_labels(labels[nu], labels[nu]) if labels is not None else None
        if D * D <= dcut:
            Us[nu] = np.eye(D * D)
            new_labels[nu] = lab
            decisions.append(AxisDecision(nu, 0, D * D, (0.0, 0.0), math.inf, False, (None, None), False))
            continue
        sides = []
        for side in (0, 1):
            E = environment(T, T, mu, nu, side)
            lam, V, lb = eigh_desc(E, lab)
            cut = choose_cut(lam, dcut, tau)
            eps = float(np.sum(np.clip(lam[cut.k:], 0.0, None)))
            sides.append((lam, V, lb, cut, eps))
        eps_b, eps_f = sides[0][4], sides[1][4]
        scale = float(np.sum(np.clip(sides[0][0], 0.0, None)))
        s = 0 if eps_b <= eps_f + SIDE_TIE * scale else 1
        lam, V, lb, cut, _ = sides[s]
        Us[nu] = V[:, : cut.k].copy()
        new_labels[nu] = None if lb is None else lb[: cut.k].copy()
        decisions.append(AxisDecision(nu, s, cut.k, (eps_b, eps_f), cut.gap, cut.flagged,
                                      (sides[0][0], sides[1][0]), True))
    return Us, new_labels, decisions


# ---------------------------------------------------------------------------
# The contraction of one step (Eqs. (2.8)-(2.9) generalised to d dimensions).
# Oracle order: slice the two output mu-legs; absorb the first transverse
# axis's isometry on both T1 legs, contract with T2 over (i2, i2', alpha),
# then absorb the remaining isometries pairwise.  Peak size D^{4(d-1)-2}.
# ---------------------------------------------------------------------------
def _leg_iso(Us: dict, nu: int, side: int) -> np.ndarray:
    """Isometry of axis nu on the merged backward (side 0) or forward (side 1)
    legs.  Us[nu] is one matrix used on both legs (the method), or a pair
    (U_backward, U_forward) -- used only by the tangent, whose product rule
    differentiates one leg at a time."""
    u = Us[nu]
    return u[side] if isinstance(u, tuple) else u


def _absorb_remaining(Y, order, t1_shape, t2_shape, Us, transverse, first):
    """Absorb U_nu for transverse[first:] pairwise on the (T1 leg, T2 leg) pairs."""
    for j, nu in enumerate(transverse[first:], start=first):
        for side in (0, 1):
            U = _leg_iso(Us, nu, side).reshape(t1_shape[2 * j], t2_shape[2 * j], -1)
            p1 = order.index(("r1", 2 * j + side))
            p2 = order.index(("r2", 2 * j + side))
            Y = np.tensordot(Y, U, axes=([p1, p2], [0, 1]))
            order = [o for o in order if o not in (("r1", 2 * j + side), ("r2", 2 * j + side))]
            order.append(("new", 2 * j + side))
    perm = [order.index(("new", i)) for i in range(2 * len(transverse))]
    return np.transpose(Y, perm)


def _step_slice(t1: np.ndarray, t2: np.ndarray, Us: dict, transverse: list, pivot: bool) -> np.ndarray:
    """t1 = T1[.., mu_b = m1, mu_f = alpha], t2 = T2[.., mu_b = alpha, mu_f = m2],
    both with legs (nu1b, nu1f, nu2b, nu2f, ..., alpha).  Returns the slice of
    the new tensor with legs (nu1, nu1', nu2, nu2', ...).

    pivot=False: contract t1 with t2 over alpha (size D^{4(d-1)}), then absorb
    every isometry pairwise.  pivot=True: first absorb the first transverse
    isometry on both legs of t1, contract with t2 over (i2, i2', alpha), then
    absorb the rest (peak size D^{4(d-1)-2}; used for large D).
    """
    nt = len(transverse)
    if nt == 0:
        return np.tensordot(t1, t2, axes=([0], [0]))
    r = 2 * nt
    if not pivot:
        Y = np.tensordot(t1, t2, axes=([t1.ndim - 1], [t2.ndim - 1]))
        order = [("r1", i) for i in range(r)] + [("r2", i) for i in range(r)]
        return _absorb_remaining(Y, order, t1.shape, t2.shape, Us, transverse, 0)
    D1, D2 = t1.shape[0], t2.shape[0]
    U0b = _leg_iso(Us, transverse[0], 0).reshape(D1, D2, -1)   # [i1, i2, new]
    U0f = _leg_iso(Us, transverse[0], 1).reshape(D1, D2, -1)
    X = np.tensordot(t1, U0b, axes=([0], [0]))           # [i1', rest1.., alpha, i2, a]
    X = np.tensordot(X, U0f, axes=([0], [0]))            # [rest1.., alpha, i2, a, i2', a']
    nr = t1.ndim - 3                                      # legs of rest1
    # contract with t2 over (i2, i2', alpha); t2 legs: [i2, i2', rest2.., alpha]
    Y = np.tensordot(X, t2, axes=([nr + 1, nr + 3, nr], [0, 1, t2.ndim - 1]))
    # Y legs: [rest1.., a, a', rest2..]
    order = ([("r1", i) for i in range(2, r)] + [("new", 0), ("new", 1)]
             + [("r2", i) for i in range(2, r)])
    return _absorb_remaining(Y, order, t1.shape, t2.shape, Us, transverse, 1)


PIVOT_ABOVE = 1 << 24      # elements of t1 . t2 above which the pivot order is used


def coarse_grain(T1: np.ndarray, T2: np.ndarray, Us: dict, mu: int, pivot: bool | None = None,
                 slices=None) -> np.ndarray:
    """New (unnormalised) tensor of a step along mu, Eqs. (2.8)-(2.9) in d dims.

    Sliced over the two output mu-legs; see _step_slice for the two orders.
    `slices` (a list of (m1, m2) pairs) computes only those output slices and
    leaves the rest zero (used to time a bounded part of a large step).
    """
    d = T1.ndim // 2
    transverse = [nu for nu in range(d) if nu != mu]
    Dm1, Dm2 = T1.shape[2 * mu], T2.shape[2 * mu + 1]
    new_dims = []
    for nu in range(d):
        if nu == mu:
            new_dims += [Dm1, Dm2]
        else:
            new_dims += [_leg_iso(Us, nu, 0).shape[1], _leg_iso(Us, nu, 1).shape[1]]
    out = np.zeros(new_dims)
    # move mu legs of T1/T2 to the front for slicing
    tl = [l for l in range(2 * d) if l not in (2 * mu, 2 * mu + 1)]
    T1m = np.ascontiguousarray(np.transpose(T1, [2 * mu, *tl, 2 * mu + 1]))  # [m1, transverse.., alpha]
    T2m = np.ascontiguousarray(np.transpose(T2, [2 * mu + 1, *tl, 2 * mu]))  # [m2, transverse.., alpha]
    if pivot is None:
        pivot = T1m[0].size * T2m[0].size // max(1, T1m.shape[-1]) > PIVOT_ABOVE
    idx = [slice(None)] * (2 * d)
    pairs = slices if slices is not None else [(m1, m2) for m1 in range(Dm1) for m2 in range(Dm2)]
    for m1, m2 in pairs:
        sl = _step_slice(T1m[m1], T2m[m2], Us, transverse, pivot)
        idx[2 * mu], idx[2 * mu + 1] = m1, m2
        out[tuple(idx)] = sl
    return out


# ---------------------------------------------------------------------------
# The flow with impurities: Eqs. (2.7)-(2.12), readings R5, R6.
# ---------------------------------------------------------------------------
@dataclass
class StepRecord:
    n: int
    axis: int
    dims: tuple
    c: float
    lnz_per_site: float
    trace: float
    m_imp: float
    nn_imp: float
    e_imp: float
    X: float
    decisions: list = field(default_factory=list)


@dataclass
class Flow:
    beta: float
    h: float
    dcut: int
    d: int
    lnz_acc: float
    T: np.ndarray
    Sm: np.ndarray
    Se: np.ndarray
    labels: list | None
    n: int = 0
    c0: float = 1.0
    records: list = field(default_factory=list)


def start(beta: float, h: float, dcut: int, d: int = 4) -> Flow:
    """Normalised initial state (a one-site torus), Eqs. (2.2), (2.6), R5."""
    T0, S0 = site_tensors(beta, h, d)
    c0 = float(np.linalg.norm(T0))
    labels = [np.array([0, 1]) for _ in range(d)] if h == 0.0 else None
    return Flow(beta, h, dcut, d, math.log(c0), T0 / c0, S0 / c0, S0 / c0, labels, 0, c0)


def observables(f: Flow, axis: int | None) -> dict:
    tr = trace(f.T)
    if not (tr > 0 and math.isfinite(tr)):
        raise FloatingPointError(f"Tr T = {tr} at n = {f.n}")
    lnz = f.lnz_acc + math.ldexp(math.log(tr), -f.n)
    m = trace(f.Sm) / tr
    nn = trace(f.Se) / tr
    X = x_indicator(f.T, axis) if axis is not None else 1.0
    return dict(lnz_per_site=lnz, trace=tr, m_imp=m, nn_imp=nn,
                e_imp=-f.d * nn - f.h * m, X=X)


def step(f: Flow, mu: int, impurities: bool = True, tau: float = TAU_DEGENERATE,
         Us_override: dict | None = None) -> StepRecord:
    """One coarse-graining step along mu of T, S_m, S_e (Eqs. (2.8)-(2.9))."""
    if Us_override is None:
        Us, new_labels, decisions = isometries(f.T, mu, f.dcut, f.labels, tau)
    else:
        Us, new_labels, decisions = Us_override, None, []
    Tn = coarse_grain(f.T, f.T, Us, mu)
    if impurities:
        Smn = coarse_grain(f.Sm, f.T, Us, mu)
        Sen = coarse_grain(f.Se, f.Se if f.n == 0 else f.T, Us, mu)
    c = float(np.linalg.norm(Tn))
    if not (c > 0 and math.isfinite(c)):
        raise FloatingPointError(f"c_n = {c} at step {f.n + 1}")
    f.n += 1
    f.T = Tn / c
    if impurities:
        f.Sm, f.Se = Smn / c, Sen / c
    f.lnz_acc += math.ldexp(math.log(c), -f.n)
    if f.labels is not None and new_labels is not None:
        f.labels = [new_labels.get(nu, f.labels[nu]) for nu in range(f.d)]
    else:
        f.labels = None
    ob = observables(f, mu) if impurities else dict(
        lnz_per_site=f.lnz_acc + math.ldexp(math.log(trace(f.T)), -f.n),
        trace=trace(f.T), m_imp=math.nan, nn_imp=math.nan, e_imp=math.nan,
        X=x_indicator(f.T, mu))
    rec = StepRecord(f.n, mu, tuple(f.T.shape[::2]), c, decisions=decisions, **ob)
    f.records.append(rec)
    return rec


def run(beta: float, h: float, dcut: int, d: int = 4, nsteps: int = 4,
        axes=None, impurities: bool = True, tau: float = TAU_DEGENERATE) -> Flow:
    """Full flow: nsteps steps cycling the axes 0, 1, .., d-1 (Sec. 2)."""
    f = start(beta, h, dcut, d)
    for n in range(nsteps):
        mu = axes[n] if axes is not None else n % d
        step(f, mu, impurities, tau)
    return f
