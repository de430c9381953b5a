"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/hotrg.h declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hotrg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hotrg_\w+)\s*\(", text)))


def test_header_declares_the_paper_calls():
    names = declared_symbols()
    for n in ("hotrg_init", "hotrg_step", "hotrg_lnZ", "hotrg_observables", "hotrg_backward"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1906_06060_amd import hotrg
    lib = hotrg.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) == set(hotrg.EXPORTS)


@pytest.mark.parametrize("beta,h,dcut", [(-0.1, 0.0, 4), (float("nan"), 0.0, 4), (0.1, float("inf"), 4),
                                          (0.1, 0.0, 0), (0.1, 0.0, 13)])
def test_init_rejects_bad_arguments_without_a_device(beta, h, dcut):
    from paper_1906_06060_amd import hotrg
    lib = hotrg.load()
    out = C.c_void_p()
    rc = lib.hotrg_init(beta, h, dcut, C.byref(out))
    assert rc == hotrg.EINVAL
    assert not out
    assert lib.hotrg_last_error()


def test_null_handles_are_rejected():
    from paper_1906_06060_amd import hotrg
    lib = hotrg.load()
    v = C.c_double()
    assert lib.hotrg_lnZ(None, C.byref(v)) == hotrg.EINVAL
    assert lib.hotrg_step(None, 0) == hotrg.EINVAL
    lib.hotrg_free(None)
