"""Forward-mode derivative of ln Z / N through the whole HOTRG flow
(TEST INFRASTRUCTURE ONLY; the reference for the GPU reverse-mode adjoint).

The flow of `oracle.hotrg` is differentiated step by step with respect to
beta or h.  Differentiating ln Z / N = sum_k 2^-k ln c_k + 2^-n ln Tr T^(n)
with every c_k held constant is exact: the step is homogeneous of degree two
in T and the isometries are scale invariant, so the normalised chain with
frozen c_k equals the unnormalised chain up to constant factors, and
d(lnZ/N) = 2^-n d Tr T^(n) / Tr T^(n).

Per step the tangent dT' collects the product rule over the two tensors and
the six isometry legs of Eqs. (2.8)-(2.9) (d-dimensional form); the isometry
tangent is the eigenvector derivative restricted to kept x discarded pairs,
  dU = V_perp (F o (V_perp^T dE U)),  F[j, i] = 1 / (lam_i - lam_j),
(rotations inside the kept space change T' only by a gauge transformation on
the new bonds and leave every trace unchanged).  Decisions (k, side) are the
forward flow's and are held fixed.
"""
from __future__ import annotations

import math

import numpy as np

from . import hotrg as H


def bond_factor_derivative(beta: float) -> np.ndarray:
    """d W / d beta for W = [[sqrt cosh b, sqrt sinh b], [sqrt cosh b, -sqrt sinh b]];
    diverges at beta = 0 through 1 / sqrt(sinh b)."""
    if not beta > 0:
        raise ValueError("the beta derivative needs beta > 0")
    c = math.sqrt(math.cosh(beta))
    s = math.sqrt(math.sinh(beta))
    dc = math.sinh(beta) / (2 * c)
    ds = math.cosh(beta) / (2 * s)
    return np.array([[dc, ds], [dc, -ds]])


def site_tensor_tangents(beta: float, h: float, d: int, wrt: str):
    """(T^(0), dT^(0)/d wrt) for the tensor of Eq. (2.2); wrt is 'beta' or 'h'."""
    W = H.bond_factor(beta)
    dW = bond_factor_derivative(beta) if wrt == "beta" else np.zeros((2, 2))
    T = np.zeros((2,) * (2 * d))
    dT = np.zeros((2,) * (2 * d))
    for row, sigma in enumerate((1.0, -1.0)):
        P, dP = W[row], dW[row]
        for _ in range(2 * d - 1):
            dP = np.multiply.outer(dP, W[row]) + np.multiply.outer(P, dW[row])
            P = np.multiply.outer(P, W[row])
        v = math.exp(beta * h * sigma)
        dv = (h if wrt == "beta" else beta) * sigma * v
        T += v * P
        dT += dv * P + v * dP
    return T, dT


def _gram_pair_tangent(T, dT, leg, other):
    rest = [l for l in range(T.ndim) if l not in (leg, other)]
    dG = np.tensordot(dT, T, axes=(rest, rest)) + np.tensordot(T, dT, axes=(rest, rest))
    if leg > other:
        dG = dG.transpose(1, 0, 3, 2)
    return dG


def environment_tangent(T, dT, mu, nu, side):
    """dE for E = environment(T, T, mu, nu, side) (product rule on both Grams)."""
    leg = 2 * nu + side
    G1 = H._gram_pair(T, leg, 2 * mu + 1)
    G2 = H._gram_pair(T, leg, 2 * mu)
    dG1 = _gram_pair_tangent(T, dT, leg, 2 * mu + 1)
    dG2 = _gram_pair_tangent(T, dT, leg, 2 * mu)
    dE = (np.einsum("pauc,qavc->pquv", dG1, G2, optimize=True)
          + np.einsum("pauc,qavc->pquv", G1, dG2, optimize=True))
    n = T.shape[leg]
    return dE.reshape(n * n, n * n)


def isometry_tangents(T, dT, mu, dcut, labels, tau=H.TAU_DEGENERATE):
    """Isometries and decisions of the forward step plus their tangents."""
    Us, new_labels, decisions = H.isometries(T, mu, dcut, labels, tau)
    dUs = {}
    for dec in decisions:
        nu = dec.nu
        if not dec.truncated:
            dUs[nu] = np.zeros_like(Us[nu])
            continue
        D = T.shape[2 * nu]
        lab = H.merged_labels(labels[nu], labels[nu]) if labels is not None else None
        E = H.environment(T, T, mu, nu, dec.side)
        lam, V, _ = H.eigh_desc(E, lab)
        k = dec.k
        U, Vp = V[:, :k], V[:, k:]
        assert np.allclose(U, Us[nu])
        dE = environment_tangent(T, dT, mu, nu, dec.side)
        F = 1.0 / (lam[None, :k] - lam[k:, None])           # F[j, i], j discarded, i kept
        dUs[nu] = Vp @ (F * (Vp.T @ dE @ U))
    return Us, dUs, new_labels, decisions


def step_tangent(T, dT, mu, dcut, labels, tau=H.TAU_DEGENERATE):
    """One step of (T, dT) -> (T'/c, dT'/c, c) with c = |T'|_F held constant."""
    Us, dUs, new_labels, decisions = isometry_tangents(T, dT, mu, dcut, labels, tau)
    Tn = H.coarse_grain(T, T, Us, mu)
    dTn = H.coarse_grain(dT, T, Us, mu) + H.coarse_grain(T, dT, Us, mu)
    for nu, dU in dUs.items():
        if not np.any(dU):
            continue
        dTn = dTn + H.coarse_grain(T, T, {**Us, nu: (dU, Us[nu])}, mu)
        dTn = dTn + H.coarse_grain(T, T, {**Us, nu: (Us[nu], dU)}, mu)
    c = float(np.linalg.norm(Tn))
    return Tn / c, dTn / c, c, new_labels, decisions


def run(beta: float, h: float, dcut: int, d: int, nsteps: int, wrt: str, axes=None,
        tau: float = H.TAU_DEGENERATE):
    """Per step n: (n, lnZ/N, d(lnZ/N)/d wrt)."""
    T0, dT0 = site_tensor_tangents(beta, h, d, wrt)
    c0 = float(np.linalg.norm(T0))
    T, dT = T0 / c0, dT0 / c0
    labels = [np.array([0, 1]) for _ in range(d)] if h == 0.0 else None
    lnz_acc = math.log(c0)
    out = []
    for n in range(1, nsteps + 1):
        mu = axes[n - 1] if axes is not None else (n - 1) % d
        T, dT, c, new_labels, _ = step_tangent(T, dT, mu, dcut, labels, tau)
        if labels is not None:
            labels = [new_labels.get(nu, labels[nu]) for nu in range(d)]
        lnz_acc += math.ldexp(math.log(c), -n)
        tr = H.trace(T)
        out.append((n, lnz_acc + math.ldexp(math.log(tr), -n), math.ldexp(H.trace(dT) / tr, -n)))
    return out
