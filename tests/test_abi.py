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
                                          (0.1, 0.0, 0), (0.1, 0.0, 14)])
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


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors of hotrg_config / hotrg_obs against the C compiler's
    # layout of the header (host gcc; no device)
    import shutil
    import subprocess
    from paper_1906_06060_amd import hotrg
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "hotrg.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(hotrg_config), offsetof(hotrg_config, eig_max_sweeps),\n'
        "         offsetof(hotrg_config, alloc), offsetof(hotrg_config, mem_budget), sizeof(hotrg_obs),\n"
        "         offsetof(hotrg_obs, block_sparse), offsetof(hotrg_config, dense_only));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(hotrg.Config), hotrg.Config.eig_max_sweeps.offset, hotrg.Config.alloc.offset,
            hotrg.Config.mem_budget.offset, C.sizeof(hotrg.Obs), hotrg.Obs.block_sparse.offset,
            hotrg.Config.dense_only.offset]
    assert got == want


@pytest.mark.parametrize("field,value", [("eig_max_sweeps", 1001), ("precision", 7)])
def test_init_ex_rejects_bad_config_without_a_device(field, value):
    from paper_1906_06060_amd import hotrg
    lib = hotrg.load()
    cfg = hotrg.Config()
    cfg.impurities = 1
    setattr(cfg, field, value)
    out = C.c_void_p()
    assert lib.hotrg_init_ex(0.1, 0.0, 4, C.byref(cfg), C.byref(out)) == hotrg.EINVAL
    assert not out


def test_init_ex_needs_alloc_and_free_together():
    from paper_1906_06060_amd import hotrg
    lib = hotrg.load()
    cfg = hotrg.Config()
    cfg.alloc = hotrg.ALLOC_FN(lambda n, ctx: None)
    out = C.c_void_p()
    assert lib.hotrg_init_ex(0.1, 0.0, 4, C.byref(cfg), C.byref(out)) == hotrg.EINVAL
    assert b"together" in lib.hotrg_last_error()
    assert not out


def test_truncate_rejects_a_null_context():
    from paper_1906_06060_amd import hotrg
    lib = hotrg.load()
    assert lib.hotrg_truncate(None, 0) == hotrg.EINVAL
