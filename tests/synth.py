"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds no HOTRG arithmetic: random tensors with the Z2 structure of the h = 0
flow (entries whose bond parities sum to odd are zero, parity of bond index i
is i mod 2), random isometries (orthonormal columns), and index samples.
"""
import numpy as np

SEED = 1906060


def z2_tensor(dims, seed=SEED, odd=False, dtype=np.float64):
    """Gaussian rank-2d tensor with legs (D0, D0, D1, D1, ..), Frobenius norm 1.

    odd=False keeps the entries with an even parity sum (a pure tensor),
    odd=True the odd ones (a one-impurity tensor)."""
    shape = []
    for D in dims:
        shape += [D, D]
    rng = np.random.default_rng(seed)
    T = rng.standard_normal(shape)
    # parity of the index sum, accumulated leg by leg with broadcasting (one
    # int8 array: no index grids of the full shape at Dcut = 12)
    par = np.zeros(shape, dtype=np.int8)
    for leg, D in enumerate(shape):
        view = [1] * len(shape)
        view[leg] = D
        par ^= (np.arange(D, dtype=np.int8) % 2).reshape(view)
    T[par != (1 if odd else 0)] = 0.0
    del par
    T /= np.linalg.norm(T)
    return T.astype(dtype, copy=False)


def isometry(n, k, seed=SEED + 1):
    """n x k matrix with orthonormal columns (QR of a Gaussian matrix)."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    return np.ascontiguousarray(q)


def sample_indices(shape, count, seed=SEED + 2):
    """`count` distinct multi-indices of `shape`, sorted, as a list of tuples."""
    rng = np.random.default_rng(seed)
    total = int(np.prod(shape))
    flat = np.sort(rng.choice(total, size=min(count, total), replace=False))
    return [tuple(int(v) for v in np.unravel_index(f, shape)) for f in flat]


def z2_isometry(D, k, seed=SEED + 3):
    """D^2 x k matrix with orthonormal columns, each column supported on the
    merged rows (i1, i2) of one parity (i1 + i2) mod 2 (parity of bond index
    i is i mod 2): the shape of an isometry of the h = 0 flow.  Columns of the
    two parities are interleaved in a random order."""
    rng = np.random.default_rng(seed)
    n = D * D
    rows = [np.array([r for r in range(n) if ((r // D) + (r % D)) % 2 == p]) for p in (0, 1)]
    k0 = min(len(rows[0]), (k + 1) // 2)
    k1 = k - k0
    if k1 > len(rows[1]):
        k1 = len(rows[1])
        k0 = k - k1
    U = np.zeros((n, k))
    cols = rng.permutation(k)
    for p, kp, cs in ((0, k0, cols[:k0]), (1, k1, cols[k0:])):
        if kp == 0:
            continue
        q, _ = np.linalg.qr(rng.standard_normal((len(rows[p]), kp)))
        U[np.ix_(rows[p], cs)] = q
    return U
