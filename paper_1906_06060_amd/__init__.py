"""MI355X-native HOTRG coarse-graining step for the 4D Ising model.

The compute lives in the HIP library libhotrg_gfx950.so (C ABI in
include/hotrg.h); `paper_1906_06060_amd.hotrg` is its ctypes binding and
`paper_1906_06060_amd.autograd` wraps ln Z / N as a torch.autograd.Function.
`paper_1906_06060_amd.tc` locates T_c(Dcut) from the X indicator and
`paper_1906_06060_amd.jump` extracts the energy and magnetisation jumps there
(Sec. 3); both drive GPU flows through the same library.
"""
from . import hotrg  # noqa: F401


def __getattr__(name):
    if name == "autograd":  # imports torch; loaded on first use
        import importlib
        return importlib.import_module(".autograd", __name__)
    raise AttributeError(name)
