"""Device-time statistics of hotrg_kernel_stats: GEMM launches and the three
phases of hotrg_step (isometries, contraction, normalisation)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1906_06060_amd import hotrg
    hotrg.load()
    return hotrg


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_phase_times_cover_the_gemm(H, precision):
    prec = H.FP64 if precision == "fp64" else H.BF16X3
    with H.Context(0.1497, 0.0, 6, precision=prec) as ctx:
        for n in range(3):
            ctx.step(n % 4)
        ctx.reset_stats()
        for n in range(3, 7):
            ctx.step(n % 4)
        ph = ctx.phase_stats()
        g = ctx.gemm_stats()
    assert ph["steps"] == 4
    assert ph["isometries_ms"] > 0 and ph["contraction_ms"] > 0 and ph["normalise_ms"] > 0
    assert 0 < g["ms"] == pytest.approx(ph["gemm_ms"])
    # the GEMMs run inside the contraction phase
    assert ph["gemm_ms"] <= ph["contraction_ms"] * 1.001 + 0.01
    assert g["flops"] > 0 and g["launches"] > 0


def test_kernel_stats_rejects_unknown_index(H):
    import ctypes as C
    with H.Context(0.1497, 0.0, 2) as ctx:
        ms, fl, ln = C.c_double(), C.c_double(), C.c_longlong()
        for k in (-1, 6):
            rc = H._lib.hotrg_kernel_stats(ctx._h, k, C.byref(ms), C.byref(ln), C.byref(fl))
            assert rc == -1
        for k in (4, 5):  # tile-scatter launches, reverse steps in the block form
            assert H._lib.hotrg_kernel_stats(ctx._h, k, C.byref(ms), C.byref(ln), C.byref(fl)) == 0
            assert ln.value == 0 and ms.value == 0.0
        ctx.reset_stats()
        assert ctx.phase_stats()["steps"] == 0
