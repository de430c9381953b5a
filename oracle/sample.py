"""Entries of one coarse-graining step straight from its definition
(TEST INFRASTRUCTURE ONLY).

For output row r = (n_nu1, n_nu2, .., m1) and column c = (n'_nu1, .., m2) the
new tensor entry of Eqs. (2.8)-(2.9) (d-dimensional form) is

  T'[n, n', .., m1, m2] = sum_{alpha, i1, i1', i2, i2', ..}
        prod_nu U_nu[(i1, i2), n_nu] U_nu[(i1', i2'), n'_nu]
        T1[i1, i1', .., m1, alpha] T2[i2, i2', .., alpha, m2].

Each row becomes a vector R1_r over (i2, i1' per axis, alpha) by absorbing
the row's isometry columns into T1; each column a vector R2_c over the same
legs from T2; the entry is their dot product.  Cost per row or column is
O(D^{2d}), so a few hundred entries are cheap at any D where T fits.
"""
from __future__ import annotations

import numpy as np


def _row_vectors(T1, Us, mu, rows):
    d = T1.ndim // 2
    transverse = [nu for nu in range(d) if nu != mu]
    tl = [l for l in range(2 * d) if l not in (2 * mu, 2 * mu + 1)]
    base = np.transpose(T1, [2 * mu, *tl, 2 * mu + 1])      # [m1, (b, f) per nu, alpha]
    out = []
    for r in rows:
        *ns, m1 = r
        R = base[m1]
        for j, nu in enumerate(transverse):
            D1 = T1.shape[2 * nu]
            u = Us[nu][:, ns[j]].reshape(D1, -1)             # [i1, i2]
            R = np.moveaxis(np.tensordot(R, u, axes=([2 * j], [0])), -1, 2 * j)
        out.append(R.reshape(-1))
    return np.array(out)


def _col_vectors(T2, Us, mu, cols):
    d = T2.ndim // 2
    transverse = [nu for nu in range(d) if nu != mu]
    tl = [l for l in range(2 * d) if l not in (2 * mu, 2 * mu + 1)]
    base = np.transpose(T2, [2 * mu + 1, *tl, 2 * mu])      # [m2, (b, f) per nu, alpha]
    out = []
    for c in cols:
        *ns, m2 = c
        R = base[m2]
        for j, nu in enumerate(transverse):
            D1 = Us[nu].shape[0] // T2.shape[2 * nu + 1]
            u = Us[nu][:, ns[j]].reshape(D1, -1)             # [i1', i2']
            R = np.moveaxis(np.tensordot(R, u, axes=([2 * j + 1], [1])), -1, 2 * j + 1)
        out.append(R.reshape(-1))
    return np.array(out)


def step_entries(T1, T2, Us: dict, mu: int, rows, cols) -> np.ndarray:
    """Matrix of new-tensor entries [len(rows), len(cols)] (unnormalised)."""
    return _row_vectors(T1, Us, mu, rows) @ _col_vectors(T2, Us, mu, cols).T


def step_entries_with_norms(T1, T2, Us: dict, mu: int, rows, cols):
    """Entries plus the Euclidean norms of each row vector and column vector
    (|entry error| of any summation order is bounded by eps * |row| |col|)."""
    R1 = _row_vectors(T1, Us, mu, rows)
    R2 = _col_vectors(T2, Us, mu, cols)
    return R1 @ R2.T, np.linalg.norm(R1, axis=1), np.linalg.norm(R2, axis=1)
