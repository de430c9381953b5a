"""The Z2 block form of the contraction (h = 0) against the oracle's dense
contraction and against the library's own dense path.

The block form splits each K slice into the two parity classes of its K
indices and never forms the parity-violating half of the output; the oracle
contracts every entry densely.  Inputs: seeded tensors with exact zeros on
their parity-violating entries (bond parity i mod 2) and isometries whose
columns each lie in one parity sector (tests/synth.py).
"""
import numpy as np
import pytest

from oracle import hotrg as OH
from oracle import sample as OS
from tests import synth
from tests.test_gpu_parity import _sampled_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1906_06060_amd import hotrg
    hotrg.load()
    return hotrg


CASES = [
    # dims, dcut, axis: ragged bond dimensions, classes of unequal size
    ((2, 2, 2, 2), 4, 0),
    ((4, 3, 2, 4), 4, 3),
    ((3, 5, 2, 4), 5, 2),
    ((1, 2, 3, 1), 3, 3),
    ((5, 4, 3, 3), 6, 1),
]


def _inputs(dims, dcut, axis, seed):
    T = synth.z2_tensor(dims, seed=seed)
    Sm = synth.z2_tensor(dims, seed=seed + 1, odd=True)
    Se = synth.z2_tensor(dims, seed=seed + 2)
    Us = {}
    for q in range(4):
        if q != axis:
            Us[q] = synth.z2_isometry(dims[q], min(dcut, dims[q] ** 2), seed=seed + 10 + q)
    return T, Sm, Se, Us


@pytest.mark.parametrize("dims,dcut,axis", CASES)
@pytest.mark.parametrize("budget", [0, 1])
def test_z2_full_tensor_fp64(H, dims, dcut, axis, budget):
    T, Sm, Se, Us = _inputs(dims, dcut, axis, 300)
    with H.Context(0.0 + 0.2, 0.0, dcut, slice_budget=budget) as ctx:
        ctx.set_state(T, Sm, Se, n=3, lnz_acc=0.0)
        ctx.step_with_isometries(axis, Us)
        ob = ctx.observables()
        got = [ctx.tensor(w) for w in range(3)]
    assert ob["block_sparse"] == 1
    want_T = OH.coarse_grain(T, T, Us, axis)
    c = np.linalg.norm(want_T)
    want = [want_T / c, OH.coarse_grain(Sm, T, Us, axis) / c, OH.coarse_grain(Se, T, Us, axis) / c]
    assert ob["last_cn"] == pytest.approx(c, rel=1e-13)
    for g, w in zip(got, want):
        assert g.shape == w.shape
        np.testing.assert_allclose(g, w, rtol=0, atol=1e-13 * max(np.abs(w).max(), 1e-300))


@pytest.mark.parametrize("dims,dcut,axis", CASES)
def test_z2_full_tensor_bf16x3(H, dims, dcut, axis):
    T, Sm, Se, Us = _inputs(dims, dcut, axis, 320)
    tv = [q for q in range(4) if q != axis]
    with H.Context(0.2, 0.0, dcut, precision=H.BF16X3, mixed_from_step=1) as ctx:
        ctx.set_state(T, Sm, Se, n=3, lnz_acc=0.0)
        ctx.step_with_isometries(axis, Us)
        ob = ctx.observables()
        got = [ctx.tensor(w) for w in range(3)]
    assert ob["block_sparse"] == 1
    cn = ob["last_cn"]
    rshape = tuple(Us[q].shape[1] for q in tv) + (dims[axis],)
    idx_all = [tuple(int(v) for v in np.unravel_index(f, rshape)) for f in range(int(np.prod(rshape)))]
    worst = 0.0
    for (T1, T2), G in zip([(T, T), (Sm, T), (Se, T)], got):
        ent, rn, cnorm = OS.step_entries_with_norms(T1, T2, Us, axis, idx_all, idx_all)
        for i, r in enumerate(idx_all):
            for j, cc in enumerate(idx_all):
                idx = [0] * 8
                for q_i, q in enumerate(tv):
                    idx[2 * q], idx[2 * q + 1] = r[q_i], cc[q_i]
                idx[2 * axis], idx[2 * axis + 1] = r[-1], cc[-1]
                scale = rn[i] * cnorm[j]
                if scale > 0:
                    worst = max(worst, abs(G[tuple(idx)] * cn - ent[i, j]) / scale)
                else:
                    assert G[tuple(idx)] == 0.0
    assert worst <= 6e-5, worst


@pytest.mark.parametrize("precision,bound", [("FP64", 1e-13), ("BF16X3", 6e-5)])
def test_z2_sampled_d8(H, precision, bound):
    _sampled_parity(H, 8, 3, getattr(H, precision), True, 24, bound, seed=71, z2=True)


def test_z2_sampled_d8_b1_slices(H):
    _sampled_parity(H, 8, 1, H.BF16X3, True, 16, 6e-5, seed=73, slice_budget=1, z2=True)


def test_z2_not_used_for_a_state_without_parity_structure(H):
    rng = np.random.default_rng(5)
    dims = (3, 3, 3, 3)
    shape = [d for D in dims for d in (D, D)]
    T = rng.standard_normal(shape)
    with H.Context(0.2, 0.0, 4, impurities=False) as ctx:
        ctx.set_state(T / np.linalg.norm(T), n=3)
        ctx.step(0)
        assert ctx.observables()["block_sparse"] == 0


@pytest.mark.parametrize("precision,rel", [("FP64", 1e-12), ("BF16X3", 1e-6)])
def test_z2_flow_equals_dense_flow(H, precision, rel):
    # the same h = 0 flow with the block form (default) and with dense_only:
    # identical dims and kept k; lnZ/N, e, X to rounding (FP64) or to the
    # bf16x3 summation-order bound; m = 0 exactly in both.  The environment
    # side (reading R2) is compared in FP64 only: mirror-symmetric states make
    # eps_b and eps_f equal up to rounding, so under bf16x3 the near-tie can
    # go either way, which changes no trace (a gauge choice)
    beta, dcut, n = 0.1497, 6, 9
    prec = getattr(H, precision)
    a = H.flow(beta, 0.0, dcut, n, precision=prec)
    b = H.flow(beta, 0.0, dcut, n, precision=prec, dense_only=True)
    assert [x["block_sparse"] for x in a] == [0] + [1] * (n - 1)
    assert all(x["block_sparse"] == 0 for x in b)
    for x, y in zip(a, b):
        assert x["dims"] == y["dims"] and x["last_k"] == y["last_k"]
        if precision == "FP64":
            assert x["last_side"] == y["last_side"]
        assert x["lnz_per_site"] == pytest.approx(y["lnz_per_site"], rel=rel)
        assert x["e_imp"] == pytest.approx(y["e_imp"], rel=100 * rel)
        assert x["X"] == pytest.approx(y["X"], rel=100 * rel)
        assert x["m_imp"] == 0.0 and y["m_imp"] == 0.0


def test_z2_flow_matches_oracle_dcut5(H):
    # whole h = 0 flow through the block form against the oracle (parity-
    # blocked eigh, dense contraction)
    beta, dcut, n = 0.1497, 5, 7
    f = OH.run(beta, 0.0, dcut, 4, n)
    got = H.flow(beta, 0.0, dcut, n)
    for g, r in zip(got, f.records):
        assert g["dims"] == r.dims
        assert g["lnz_per_site"] == pytest.approx(r.lnz_per_site, rel=1e-10)
        assert g["nn_imp"] == pytest.approx(r.nn_imp, rel=1e-8)
        assert g["X"] == pytest.approx(r.X, rel=1e-8)
        assert g["m_imp"] == 0.0
    assert sum(g["block_sparse"] for g in got) == n - 1


@pytest.mark.parametrize("budget", [0, 1])
def test_z2_tile_scatter_bitwise_equals_element_scatter(H, monkeypatch, budget):
    # The tile form of the last products' Z2 scatter (outputs gathered in LDS,
    # written as whole 16-byte pieces) computes every operand entry with the
    # same arithmetic in the same order as the element-wise scatter, and puts
    # it at the same place: the bf16x3 flows must agree bit for bit, with and
    # without K slices that fix b1'.
    beta, dcut, n = 0.1497, 6, 8

    def run():
        out = []
        with H.Context(beta, 0.0, dcut, precision=H.BF16X3, slice_budget=budget) as ctx:
            for k in range(n):
                ctx.step(k % 4)
                out.append(ctx.observables())
            tiles = ctx.z2_tile_launches()
            tensors = [ctx.tensor(w) for w in range(3)]
        return out, tiles, tensors

    monkeypatch.setenv("HOTRG_Z2_TILE", "1")
    a, ta, Ta = run()
    monkeypatch.setenv("HOTRG_Z2_TILE", "0")
    b, tb, Tb = run()
    assert ta > 0 and tb == 0
    for x, y in zip(a, b):
        assert x["block_sparse"] == y["block_sparse"]
        for key in ("lnz_per_site", "nn_imp", "X", "last_cn"):
            assert x[key] == y[key], key
        assert x["m_imp"] == 0.0 and y["m_imp"] == 0.0
    for u, v in zip(Ta, Tb):
        np.testing.assert_array_equal(u, v)
