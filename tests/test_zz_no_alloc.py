"""hotrg_observables_noalloc (no device allocation: a fixed per-GPU scratch
array) against hotrg_observables on the same states, through the C ABI: two
calls in a row, the second on a smaller state."""
import math

import numpy as np
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


def _state(H, dcut, nsteps, h):
    import torch
    with H.Context(0.1497, h, dcut) as ctx:
        for n in range(nsteps):
            ctx.step(n % 4)
        ob = ctx.observables()
        dev = [torch.from_numpy(ctx.tensor(w)).cuda() for w in range(3)]
    torch.cuda.synchronize()
    return ob, dev


def test_noalloc_observables_equal_the_context_call(H):
    import torch
    big = _state(H, 8, 6, 1e-4)      # dims 8^4, X along axis 1
    small = _state(H, 4, 3, 0.0)     # dims (4, 4, 4, 3)-like, h = 0
    for (ob, dev), h in ((big, 1e-4), (small, 0.0)):
        assert tuple(ob["dims"]) == tuple(dev[0].shape[::2])
        before = torch.cuda.memory_allocated()
        got = H.observables_noalloc(dev[0].data_ptr(), ob["dims"], ob["last_axis"], h=h, n=ob["n"],
                                    lnz_acc=0.0, Sm_ptr=dev[1].data_ptr(), Se_ptr=dev[2].data_ptr())
        assert torch.cuda.memory_allocated() == before
        # same kernels and host arithmetic: bitwise equal
        for key in ("trace", "m_imp", "nn_imp", "e_imp", "X"):
            assert got[key] == ob[key], key
        assert got["dims"] == ob["dims"] and got["n"] == ob["n"] and got["last_axis"] == ob["last_axis"]
        assert got["lnz_per_site"] == math.ldexp(math.log(ob["trace"]), -ob["n"])
        # pure tensor only: impurity ratios undefined
        pure = H.observables_noalloc(dev[0].data_ptr(), ob["dims"], ob["last_axis"], n=ob["n"])
        assert pure["X"] == ob["X"] and math.isnan(pure["m_imp"])


def test_noalloc_rejects_dims_above_the_scratch(H):
    import torch
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HotrgError) as e:
        H.observables_noalloc(x.data_ptr(), (14, 1, 1, 1), 0)
    assert e.value.code == H.EINVAL and "1..13" in str(e.value)
