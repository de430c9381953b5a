"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test names the property it checks and why a plausible mistake in the
oracle (a dropped term, a wrong sign or index, a transposed operand) would
fail it.  No GPU involved.
"""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import hotrg as H


# --- initial tensors (Sec. 2, Eqs. (2.1), (2.2), (2.6)) ---------------------
@pytest.mark.parametrize("beta", [0.0, 0.05, 0.1497, 0.7])
def test_bond_factor_reproduces_bond_matrix(beta):
    W = H.bond_factor(beta)
    want = np.array([[math.exp(beta), math.exp(-beta)], [math.exp(-beta), math.exp(beta)]])
    np.testing.assert_allclose(W @ W.T, want, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("beta,h", [(0.1497, 0.0), (0.3, 0.2), (0.05, -0.7)])
def test_trace_of_initial_tensor_is_one_site_torus(d, beta, h):
    # one site with a self-bond on every axis: Z = sum_s e^{d beta} e^{beta h s}
    T, S = H.site_tensors(beta, h, d)
    assert H.trace(T) == pytest.approx(2 * math.exp(d * beta) * math.cosh(beta * h), rel=1e-14)
    assert H.trace(S) / H.trace(T) == pytest.approx(math.tanh(beta * h), rel=1e-13, abs=1e-15)


def test_initial_tensor_odd_entries_vanish_at_zero_field():
    T, S = H.site_tensors(0.2, 0.0, 4)
    idx = np.indices(T.shape).sum(axis=0) % 2
    assert np.all(T[idx == 1] == 0.0)
    assert np.all(S[idx == 0] == 0.0)


# --- environments: Gram form equals M M^T ----------------------------------
@pytest.mark.parametrize("d,mu,nu,side", [(2, 1, 0, 0), (2, 0, 1, 1), (3, 2, 0, 1), (3, 0, 2, 0),
                                          (4, 3, 1, 0), (4, 0, 2, 1)])
def test_environment_gram_form_matches_materialised_product(d, mu, nu, side):
    rng = np.random.default_rng(17 + d + 3 * mu + nu)
    shape = []
    for ax in range(d):
        D = 2 if d == 4 else 3
        shape += [D, D]
    T1 = rng.standard_normal(shape)
    T2 = rng.standard_normal(shape)
    E = H.environment(T1, T2, mu, nu, side)
    Ed = H.environment_direct(T1, T2, mu, nu, side)
    np.testing.assert_allclose(E, Ed, rtol=1e-12, atol=1e-12 * np.abs(Ed).max())


# --- exact results that an untruncated flow must reproduce -------------------
@pytest.mark.parametrize("beta,h", [(0.3, 0.0), (0.7, 0.2), (1.1, -0.05)])
def test_d1_flow_equals_transfer_matrix(beta, h):
    f = H.run(beta, h, dcut=4, d=1, nsteps=6)
    for r in f.records:
        assert r.lnz_per_site == pytest.approx(X.transfer_1d(beta, h, 2 ** r.n), rel=1e-13)


@pytest.mark.parametrize("L,steps", [((2, 1), 1), ((2, 2), 2), ((4, 2), 3), ((4, 4), 4)])
@pytest.mark.parametrize("beta,h", [(0.44, 0.0), (0.3, 0.1), (0.6, -0.02)])
def test_d2_untruncated_flow_equals_enumeration(L, steps, beta, h):
    f = H.run(beta, h, dcut=256, d=2, nsteps=steps)
    b = X.brute_force(beta, h, L)
    r = f.records[-1]
    assert r.lnz_per_site == pytest.approx(b["lnz_per_site"], rel=1e-13)
    assert r.m_imp == pytest.approx(b["m"], rel=1e-12, abs=1e-14)
    assert r.nn_imp == pytest.approx(b["nn"], rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("L,steps", [((2, 1, 1), 1), ((2, 2, 1), 2), ((2, 2, 2), 3)])
@pytest.mark.parametrize("beta,h", [(0.22, 0.0), (0.25, 0.15)])
def test_d3_untruncated_flow_equals_enumeration(L, steps, beta, h):
    f = H.run(beta, h, dcut=256, d=3, nsteps=steps)
    b = X.brute_force(beta, h, L)
    r = f.records[-1]
    assert r.lnz_per_site == pytest.approx(b["lnz_per_site"], rel=1e-13)
    assert r.m_imp == pytest.approx(b["m"], rel=1e-12, abs=1e-14)
    assert r.nn_imp == pytest.approx(b["nn"], rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("L,steps", [((2, 1, 1, 1), 1), ((2, 2, 1, 1), 2)])
@pytest.mark.parametrize("beta,h", [(0.1497, 0.0), (0.2, 0.1), (0.12, -0.3)])
def test_d4_untruncated_flow_equals_enumeration(L, steps, beta, h):
    f = H.run(beta, h, dcut=256, d=4, nsteps=steps)
    b = X.brute_force(beta, h, L)
    r = f.records[-1]
    assert r.lnz_per_site == pytest.approx(b["lnz_per_site"], rel=1e-13)
    assert r.m_imp == pytest.approx(b["m"], rel=1e-12, abs=1e-14)
    assert r.nn_imp == pytest.approx(b["nn"], rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("beta,h", [(0.1497, 0.0), (0.2, 0.07)])
def test_d4_eight_site_torus_via_trace_of_last_step(beta, h):
    # 2x2x2x1: steps 1-2 untruncated, the third (along z) fused with the
    # trace: Tr T' = Tr(P P), P[z, z'] = sum_{x,y,t} T2[x,x,y,y,z,z',t,t]
    f = H.run(beta, h, dcut=256, d=4, nsteps=2)
    T = f.T
    P = np.einsum("aabbzctt->zc", T)
    # T = T_unnorm / lam with ln lam = 4 lnz_acc; Z_8 = lam^2 Tr(P P)
    lnz = f.lnz_acc + math.log(np.trace(P @ P)) / 8
    b = X.brute_force(beta, h, (2, 2, 2, 1))
    assert lnz == pytest.approx(b["lnz_per_site"], rel=1e-13)


@pytest.mark.parametrize("d,L,steps,axis", [(2, (2, 2), 2, 1), (2, (4, 2), 3, 0), (4, (2, 2, 1, 1), 2, 1)])
def test_x_indicator_is_ratio_of_torus_partition_functions(d, L, steps, axis):
    # untruncated: A is the transfer matrix of the block along `axis`, so
    # (Tr A)^2 / Tr A^2 = Z(L)^2 / Z(L with that extent doubled)
    beta, h = 0.37, 0.05
    f = H.run(beta, h, dcut=256, d=d, nsteps=steps)
    Xv = f.records[-1].X
    L2 = list(L)
    L2[axis] *= 2
    z1 = X.brute_force(beta, h, L)
    z2 = X.brute_force(beta, h, tuple(L2))
    want = math.exp(2 * z1["lnz_per_site"] * z1["N"] - z2["lnz_per_site"] * z2["N"])
    assert Xv == pytest.approx(want, rel=1e-12)


# --- special cases of the truncated flow ------------------------------------
@pytest.mark.parametrize("h", [0.0, 0.4])
@pytest.mark.parametrize("dcut", [2, 4])
def test_beta_zero_gives_ln2_at_every_step(h, dcut):
    f = H.run(0.0, h, dcut=dcut, d=4, nsteps=10)
    for r in f.records:
        assert r.lnz_per_site == pytest.approx(math.log(2.0), abs=1e-14)
    assert f.records[-1].dims == (1, 1, 1, 1)


@pytest.mark.parametrize("beta", [0.01, 0.02])
def test_d4_high_temperature_leading_terms(beta):
    # lnZ/N = ln 2 + d ln cosh b + (d(d-1)/2) t^4 + O(t^6).  Truncation at a
    # small Dcut removes part of the t^4 plaquette term (a truncation effect,
    # not an oracle defect), so only the leading terms are pinned: a wrong W
    # or a dropped bond would miss by O(t^2).
    f = H.run(beta, 0.0, dcut=4, d=4, nsteps=16, impurities=False)
    t = math.tanh(beta)
    rest = f.records[-1].lnz_per_site - math.log(2.0) - 4 * math.log(math.cosh(beta))
    assert 0.0 < rest < 6 * t ** 4


def test_d3_high_temperature_truncation_error_falls_with_dcut():
    beta = 0.02
    errs = []
    for dcut in (4, 6, 8):
        f = H.run(beta, 0.0, dcut=dcut, d=3, nsteps=15, impurities=False)
        errs.append(abs(f.records[-1].lnz_per_site - X.high_t_lnz(beta, 3)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.2 * 3 * math.tanh(beta) ** 4


def test_z2_symmetry():
    f0 = H.run(0.16, 0.0, dcut=4, d=4, nsteps=8)
    for r in f0.records:
        assert r.m_imp == 0.0
    fp = H.run(0.14, 0.01, dcut=4, d=4, nsteps=8)
    fm = H.run(0.14, -0.01, dcut=4, d=4, nsteps=8)
    for a, b in zip(fp.records, fm.records):
        assert a.lnz_per_site == pytest.approx(b.lnz_per_site, rel=1e-13)
        assert a.m_imp == pytest.approx(-b.m_imp, rel=1e-10)
        assert a.nn_imp == pytest.approx(b.nn_imp, rel=1e-10)


# --- d = 2 infinite lattice: truncation-limited convergence to Onsager -------
@pytest.mark.parametrize("beta", [0.35, 0.55])
def test_d2_converges_to_onsager(beta):
    exact = X.onsager_lnz(beta)
    errs = []
    for dcut in (8, 16):
        f = H.run(beta, 0.0, dcut=dcut, d=2, nsteps=32)
        errs.append(abs(f.records[-1].lnz_per_site - exact))
    assert errs[1] < 0.05 * errs[0]
    assert errs[1] < 1e-8
    e_imp = f.records[-1].e_imp
    assert e_imp == pytest.approx(X.onsager_energy(beta), abs=2e-5)


def test_d2_energy_sign_and_relation():
    # e = -d <ss> - h m (reading R8), and <ss> in (0, 1) for beta > 0
    f = H.run(0.3, 0.05, dcut=8, d=2, nsteps=12)
    r = f.records[-1]
    assert 0 < r.nn_imp < 1
    assert r.e_imp == pytest.approx(-2 * r.nn_imp - 0.05 * r.m_imp, rel=1e-15)


# --- truncation rule (R3) ---------------------------------------------------
def test_cut_drops_back_out_of_degenerate_multiplet():
    lam = np.array([1.0, 0.5, 0.2, 0.2, 0.1])
    c = H.choose_cut(lam, 3)
    assert c.k == 2 and not c.flagged
    c = H.choose_cut(lam, 4)
    assert c.k == 4
    lam = np.array([1.0, 1.0, 1.0, 0.1])
    c = H.choose_cut(lam, 2)
    assert c.flagged and c.k == 2
    assert H.choose_cut(lam, 4).k == 4


def test_parity_blocked_eigh_matches_dense_spectrum():
    rng = np.random.default_rng(5)
    lab = np.array([0, 1, 1, 0, 0, 1])
    A = rng.standard_normal((6, 6))
    E = A @ A.T
    E[lab[:, None] != lab[None, :]] = 0.0
    lam, V, lb = H.eigh_desc(E, lab)
    np.testing.assert_allclose(lam, np.sort(np.linalg.eigvalsh(E))[::-1], rtol=1e-13)
    np.testing.assert_allclose(V @ np.diag(lam) @ V.T, E, atol=1e-12)
    for j in range(6):
        assert np.all(V[lab != lb[j], j] == 0.0)


# --- the contraction itself against a direct sum over every index ----------
@pytest.mark.parametrize("pivot", [False, True])
def test_contraction_matches_full_einsum_d4(pivot):
    rng = np.random.default_rng(11)
    D = 2
    T1 = rng.standard_normal((D,) * 8)
    T2 = rng.standard_normal((D,) * 8)
    Us = {nu: np.linalg.qr(rng.standard_normal((D * D, 3)))[0] for nu in (0, 1, 2)}
    out = H.coarse_grain(T1, T2, Us, 3, pivot=pivot)
    Ux, Uy, Uz = (Us[i].reshape(D, D, 3) for i in range(3))
    want = np.einsum("abcdefgz,hijklmzq,ahA,biB,cjC,dkD,elE,fmF->ABCDEFgq",
                     T1, T2, Ux, Ux, Uy, Uy, Uz, Uz, optimize=True)
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("pivot", [False, True])
def test_both_contraction_orders_agree_on_a_truncated_d4_step(pivot):
    f = H.run(0.1497, 0.02, dcut=4, d=4, nsteps=3)
    Us, _, _ = H.isometries(f.T, 3, 4, None)
    a = H.coarse_grain(f.T, f.T, Us, 3, pivot=pivot)
    b = H.coarse_grain(f.T, f.T, Us, 3, pivot=not pivot)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-13 * np.abs(a).max())


# --- entry sampler: an independent route to single entries ------------------
@pytest.mark.parametrize("mu", [0, 3])
def test_sampled_entries_match_full_step(mu):
    from oracle import sample
    from tests import synth
    T1 = synth.z2_tensor((3, 3, 2, 3), seed=1)
    T2 = synth.z2_tensor((3, 3, 2, 3), seed=2)
    dims = T1.shape[::2]
    Us = {nu: synth.isometry(dims[nu] ** 2, min(4, dims[nu] ** 2), seed=10 + nu) for nu in range(4) if nu != mu}
    full = H.coarse_grain(T1, T2, Us, mu)
    tv = [nu for nu in range(4) if nu != mu]
    rshape = tuple(Us[nu].shape[1] for nu in tv) + (dims[mu],)
    rows = synth.sample_indices(rshape, 7, seed=3)
    cols = synth.sample_indices(rshape, 5, seed=4)
    got = sample.step_entries(T1, T2, Us, mu, rows, cols)
    for i, r in enumerate(rows):
        for j, c in enumerate(cols):
            idx = [0] * 8
            for q, nu in enumerate(tv):
                idx[2 * nu], idx[2 * nu + 1] = r[q], c[q]
            idx[2 * mu], idx[2 * mu + 1] = r[-1], c[-1]
            assert got[i, j] == pytest.approx(full[tuple(idx)], rel=1e-12, abs=1e-15)


# --- forward-mode tangent (reference for the reverse-mode adjoint) ----------
@pytest.mark.parametrize("d,L,steps", [(2, (4, 4), 4), (3, (2, 2, 2), 3), (4, (2, 2, 1, 1), 2)])
@pytest.mark.parametrize("beta,h", [(0.3, 0.1), (0.25, 0.0)])
def test_tangent_equals_brute_force_derivatives(d, L, steps, beta, h):
    from oracle import tangent as TG
    b = X.brute_force(beta, h, L)
    assert TG.run(beta, h, 256, d, steps, "beta")[-1][2] == pytest.approx(b["dlnz_dbeta"], rel=1e-12)
    assert TG.run(beta, h, 256, d, steps, "h")[-1][2] == pytest.approx(b["dlnz_dh"], rel=1e-11, abs=1e-15)


@pytest.mark.parametrize("wrt", ["beta", "h"])
def test_tangent_agrees_with_central_differences_on_a_truncated_flow(wrt):
    # the FD error is O(delta^2): it must shrink ~100x from delta = 1e-4 to 1e-5
    from oracle import tangent as TG
    beta, h, D, n = 0.1497, 0.02, 4, 6
    dl = TG.run(beta, h, D, 4, n, wrt)[-1][2]
    errs = []
    for delta in (1e-4, 1e-5):
        bp, hp = (beta + delta, h) if wrt == "beta" else (beta, h + delta)
        bm, hm = (beta - delta, h) if wrt == "beta" else (beta, h - delta)
        fp = H.run(bp, hp, D, 4, n, impurities=False).records[-1].lnz_per_site
        fm = H.run(bm, hm, D, 4, n, impurities=False).records[-1].lnz_per_site
        errs.append(abs(dl - (fp - fm) / (2 * delta)) / abs(dl))
    assert errs[1] < 1e-6
    # (at delta = 1e-5 rounding of lnZ, ~1e-16 / delta, starts to show for the small h derivative)
    assert errs[1] < errs[0] / 10 or errs[1] < 1e-8


def test_site_tensor_tangent_matches_differences():
    from oracle import tangent as TG
    for wrt in ("beta", "h"):
        T, dT = TG.site_tensor_tangents(0.2, 0.3, 4, wrt)
        e = 1e-6
        Tp, _ = H.site_tensors(0.2 + (e if wrt == "beta" else 0), 0.3 + (e if wrt == "h" else 0), 4)
        Tm, _ = H.site_tensors(0.2 - (e if wrt == "beta" else 0), 0.3 - (e if wrt == "h" else 0), 4)
        np.testing.assert_allclose(dT, (Tp - Tm) / (2 * e), rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------------------
# T_c(Dcut) from the X indicator (Sec. 3): the d = 2 flow pins the bisection
# to Onsager's exact critical coupling; deep in each phase X takes its limit.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beta,limit", [(0.30, 1.0), (0.60, 2.0)])
def test_x_indicator_limits_in_each_phase(beta, limit):
    from oracle import tc
    assert tc.final_x(beta, 8, 2, 30) == pytest.approx(limit, abs=1e-3)


def test_d2_x_bisection_brackets_onsager_beta_c():
    from oracle import tc
    beta_c = 0.5 * math.log(1.0 + math.sqrt(2.0))
    r = tc.bisect(8, 2, 0.40, 0.48, 14, 40)
    assert r["beta_hi"] - r["beta_lo"] == pytest.approx(0.08 / 2 ** 14)
    mid = 0.5 * (r["beta_lo"] + r["beta_hi"])
    assert abs(mid - beta_c) / beta_c < 5e-4
    # every point on the ordered side of the final bracket has X near 2, on
    # the disordered side X below the threshold
    for b, x in r["points"]:
        assert (x > 1.5) == (b >= r["beta_hi"])


# ---------------------------------------------------------------------------
# Energy and magnetisation jumps (Sec. 3): the zero-field limit of m against
# Onsager's spontaneous magnetisation, and the two-sided straight-line jumps
# against the same lines drawn through Onsager's closed forms.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beta,rel", [(0.5, 1e-4), (0.6, 1e-6)])
def test_zero_field_magnetisation_equals_onsager(beta, rel):
    from oracle import jump
    m0, m1, m2 = jump.spontaneous_m(beta, 8, 2, 40)
    assert m0 == pytest.approx(X.onsager_magnetization(beta), rel=rel)


def test_zero_field_magnetisation_vanishes_when_disordered():
    from oracle import jump
    m0, m1, m2 = jump.spontaneous_m(0.40, 8, 2, 40)
    assert m1 > 1e-10 and m2 == pytest.approx(2 * m1, rel=1e-6)
    assert abs(m0) < 1e-3 * m1


def test_d2_two_sided_lines_match_onsager_lines():
    from oracle import jump
    t_c = 2.0 / math.log(1.0 + math.sqrt(2.0))
    temps = [1.8, 1.9, 2.6, 2.7]
    r = jump.jumps(8, 2, t_c, temps, 40)

    def at_tc(ts, ys):
        a, b = np.polyfit(ts, ys, 1)
        return a * t_c + b

    e = [X.onsager_energy(1.0 / T) for T in temps]
    m = [X.onsager_magnetization(1.0 / T) if T < t_c else 0.0 for T in temps]
    assert r["delta_e"] == pytest.approx(at_tc(temps[2:], e[2:]) - at_tc(temps[:2], e[:2]), abs=5e-3)
    assert r["delta_m"] == pytest.approx(at_tc(temps[:2], m[:2]) - at_tc(temps[2:], m[2:]), abs=1e-4)


# ---------------------------------------------------------------------------
# Regression guard (not a pin): the oracle still reproduces the stored flow
# of tests/golden/, which tests/golden/make_golden.py wrote from it.
# ---------------------------------------------------------------------------
def test_oracle_reproduces_stored_dcut4_flow():
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "dcut4_beta01497_16steps.json")))
    f = H.run(gold["beta"], gold["h"], gold["dcut"], 4, len(gold["steps"]))
    for r, w in zip(f.records, gold["steps"]):
        assert list(r.dims) == w["dims"]
        assert r.lnz_per_site == pytest.approx(w["lnz_per_site"], rel=1e-12)
        assert r.e_imp == pytest.approx(w["e_imp"], abs=1e-10)
        assert r.X == pytest.approx(w["X"], abs=1e-10)
        assert r.m_imp == w["m_imp"]
