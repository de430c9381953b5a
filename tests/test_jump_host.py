"""Host logic of the jump extraction (paper_1906_06060_amd.jump) on
constructed points; the GPU flows it drives are covered in test_gpu_jump.py."""
import pytest

from paper_1906_06060_amd import jump


def test_zero_field_limit_of_a_line():
    assert jump.zero_field_limit(3.0 + 2e-9 * 5, 3.0 + 4e-9 * 5, 2e-9, 4e-9) == pytest.approx(3.0, abs=1e-15)
    with pytest.raises(ValueError):
        jump.zero_field_limit(1.0, 2.0, 1e-9, 1e-9)


def test_line_value_is_least_squares():
    # exact line, then a symmetric perturbation that leaves the fit unchanged
    assert jump.line_value([1.0, 2.0, 3.0], [2.0, 4.0, 6.0], 10.0) == pytest.approx(20.0)
    assert jump.line_value([1.0, 2.0, 3.0], [2.1, 3.8, 6.1], 2.0) == pytest.approx(4.0)
    with pytest.raises(ValueError):
        jump.line_value([1.0], [1.0], 2.0)
    with pytest.raises(ValueError):
        jump.line_value([1.0, 1.0], [1.0, 2.0], 2.0)


def test_jumps_from_points_sides_and_signs():
    # e: -1 + 0.1 T below, -0.5 + 0.1 T above; m: 0.8 - 0.2 T below, 0 above
    pts = [{"T": T, "e": (-1.0 if T < 5 else -0.5) + 0.1 * T, "m": (0.8 - 0.02 * T) if T < 5 else 0.0}
           for T in (4.0, 4.5, 5.5, 6.0)]
    r = jump.jumps_from_points(pts, 5.0)
    assert r["delta_e"] == pytest.approx(0.5)
    assert r["delta_m"] == pytest.approx(0.7)
    assert r["e_below"] == pytest.approx(-0.5) and r["e_above"] == pytest.approx(0.0)
