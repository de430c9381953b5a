"""Host logic of the T_c bisection (paper_1906_06060_amd.tc) with a synthetic
X(beta); the GPU flows it normally drives are covered in test_gpu_tc.py."""
import pytest

from paper_1906_06060_amd import tc


def _step_x(beta_c):
    return lambda b: 2.0 if b > beta_c else 1.0


def test_bisection_brackets_the_jump():
    r = tc.bisect_transition(_step_x(0.1234567), 0.10, 0.20, 20)
    assert r["beta_lo"] <= 0.1234567 < r["beta_hi"]
    assert r["beta_hi"] - r["beta_lo"] == pytest.approx(0.1 / 2 ** 20)
    assert len(r["points"]) == 22 and r["unsettled"] == 0
    assert r["T_c"] == pytest.approx(1 / 0.1234567, rel=1e-5)


def test_bisection_rejects_a_bracket_without_transition():
    with pytest.raises(ValueError):
        tc.bisect_transition(_step_x(0.3), 0.10, 0.20, 5)
    with pytest.raises(ValueError):
        tc.bisect_transition(_step_x(0.05), 0.10, 0.20, 5)
    with pytest.raises(ValueError):
        tc.bisect_transition(_step_x(0.15), 0.20, 0.10, 5)


def test_unsettled_points_are_counted_and_phase_uses_the_midpoint():
    xs = {0.1: 1.0, 0.2: 2.0, 0.15: 1.6, 0.125: 1.3}
    r = tc.bisect_transition(lambda b: xs[round(b, 6)], 0.1, 0.2, 2)
    assert (r["beta_lo"], r["beta_hi"]) == pytest.approx((0.125, 0.15))
    assert r["unsettled"] == 2
    with pytest.raises(ValueError):
        tc.phase(float("nan"))


def test_scan_finds_first_disordered_to_ordered_pair():
    pair, pts = tc.bracket_by_scan(_step_x(0.147), [0.150, 0.144, 0.146, 0.148])
    assert pair == (0.146, 0.148)
    pair, pts = tc.bracket_by_scan(_step_x(0.2), [0.1, 0.15])
    assert pair is None and len(pts) == 2
