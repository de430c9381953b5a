"""Closed forms and brute force that pin the HOTRG oracle (TEST INFRASTRUCTURE ONLY).

None of this is the HOTRG method; each function is an independent route to a
quantity that an exact (untruncated) or well-converged HOTRG flow must
reproduce.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.special import ellipk


def brute_force(beta: float, h: float, L: tuple) -> dict:
    """Enumerate every spin configuration of a periodic d-torus (Eq. (2.1)).

    Bond convention of the tensor network (Eq. (2.3), periodic boundary):
    each site i carries exactly one bond per axis to i + e_axis (mod L_axis).
    L = 1 gives a self-bond (factor e^beta), L = 2 a doubled bond.
    Returns lnZ/N, <sigma_0>, and <sigma_0 sigma_{0+e_0}> (pair along axis 0).
    """
    L = tuple(int(x) for x in L)
    d = len(L)
    sites = list(itertools.product(*[range(l) for l in L]))
    index = {s: i for i, s in enumerate(sites)}
    N = len(sites)
    if N > 20:
        raise ValueError("too many spins for enumeration")
    bonds = []
    for s in sites:
        for ax in range(d):
            t = list(s)
            t[ax] = (t[ax] + 1) % L[ax]
            bonds.append((index[s], index[tuple(t)]))
    bi = np.array([b[0] for b in bonds])
    bj = np.array([b[1] for b in bonds])
    confs = np.array(list(itertools.product((1.0, -1.0), repeat=N)))     # [2^N, N]
    energy = beta * np.sum(confs[:, bi] * confs[:, bj], axis=1) + beta * h * np.sum(confs, axis=1)
    emax = energy.max()
    w = np.exp(energy - emax)
    Z = w.sum()
    lnz = (math.log(Z) + emax) / N
    m = float(np.sum(w * confs[:, 0]) / Z)
    pair = index[tuple((1 % L[0]) if k == 0 else 0 for k in range(d))]
    nn = float(np.sum(w * confs[:, 0] * confs[:, pair]) / Z)
    # per-site derivatives of lnZ / N: d/dbeta = <sum_bonds s s + h sum s> / N,
    # d/dh = beta <sum s> / N
    bond_sum = np.sum(confs[:, bi] * confs[:, bj], axis=1)
    spin_sum = np.sum(confs, axis=1)
    dbeta = float(np.sum(w * (bond_sum + h * spin_sum)) / Z) / N
    dh = beta * float(np.sum(w * spin_sum) / Z) / N
    return dict(lnz_per_site=lnz, m=m, nn=nn, N=N, dlnz_dbeta=dbeta, dlnz_dh=dh)


def transfer_1d(beta: float, h: float, N: int) -> float:
    """lnZ/N of the periodic Ising chain: Z = l+^N + l-^N."""
    a = math.exp(beta) * math.cosh(beta * h)
    r = math.sqrt(math.exp(2 * beta) * math.sinh(beta * h) ** 2 + math.exp(-2 * beta))
    lp, lm = a + r, a - r
    return (N * math.log(lp) + math.log1p((lm / lp) ** N)) / N


BETA_C_2D = 0.5 * math.log(1.0 + math.sqrt(2.0))


def onsager_lnz(beta: float, n: int = 2000) -> float:
    """Onsager's free energy of the infinite square lattice (h = 0):
    lnZ/N = ln 2 + (1/8 pi^2) int int ln[cosh^2 2b - sinh 2b (cos t1 + cos t2)]
    over [0, 2pi]^2.  The integrand is periodic and smooth away from beta_c,
    so the midpoint rule converges exponentially in n."""
    t = (np.arange(n) + 0.5) * (2 * math.pi / n)
    c1 = np.cos(t)[:, None]
    c2 = np.cos(t)[None, :]
    ch = math.cosh(2 * beta) ** 2
    sh = math.sinh(2 * beta)
    val = np.log(ch - sh * (c1 + c2)).mean() * 4 * math.pi ** 2
    return math.log(2.0) + val / (8 * math.pi ** 2)


def onsager_energy(beta: float) -> float:
    """e = -(1/N) dlnZ/dbeta = -coth 2b [1 + (2/pi)(2 tanh^2 2b - 1) K(k)],
    k = 2 sinh 2b / cosh^2 2b (scipy's ellipk takes m = k^2)."""
    k = 2 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    K = ellipk(k * k)
    return -(1.0 / math.tanh(2 * beta)) * (1 + (2 / math.pi) * (2 * math.tanh(2 * beta) ** 2 - 1) * K)


def onsager_magnetization(beta: float) -> float:
    """Spontaneous magnetisation (1 - sinh^-4 2b)^(1/8) for beta > beta_c."""
    if beta <= BETA_C_2D:
        return 0.0
    return (1.0 - math.sinh(2 * beta) ** -4) ** 0.125


def high_t_lnz(beta: float, d: int) -> float:
    """High-temperature series of the infinite hypercubic lattice at h = 0:
    lnZ/N = ln 2 + d ln cosh b + (d(d-1)/2) tanh^4 b + O(tanh^6 b)
    (d(d-1)/2 elementary plaquettes per site)."""
    t = math.tanh(beta)
    return math.log(2.0) + d * math.log(math.cosh(beta)) + d * (d - 1) / 2 * t ** 4
