"""ctypes binding of the HOTRG C ABI (include/hotrg.h).

Argument marshalling only: every step of the method runs in the HIP library.
The library must be built (``python -m paper_1906_06060_amd.build``); there is
no fallback of any kind -- a missing library raises ``HotrgUnavailable``.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhotrg_gfx950.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5
FP64, BF16X3 = 0, 1

# every symbol declared in include/hotrg.h
EXPORTS = (
    "hotrg_init", "hotrg_init_ex", "hotrg_step", "hotrg_lnZ", "hotrg_observables",
    "hotrg_backward", "hotrg_free", "hotrg_last_error", "hotrg_get_dims", "hotrg_get_tensor",
    "hotrg_set_state", "hotrg_truncate", "hotrg_step_with_isometries", "hotrg_get_isometry",
    "hotrg_get_spectrum", "hotrg_kernel_stats", "hotrg_reset_stats", "hotrg_observables_noalloc",
)

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class HotrgUnavailable(RuntimeError):
    pass


class HotrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hotrg error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("precision", C.c_int),
        ("impurities", C.c_int),
        ("keep_checkpoints", C.c_int),
        ("mixed_from_step", C.c_int),
        ("tau_deg", C.c_double),
        ("stream", C.c_void_p),
        ("slice_budget", C.c_size_t),
        ("eig_max_sweeps", C.c_int),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("alloc_ctx", C.c_void_p),
        ("mem_budget", C.c_size_t),
        ("dense_only", C.c_int),
    ]


class Obs(C.Structure):
    _fields_ = [
        ("n", C.c_int),
        ("dims", C.c_int * 4),
        ("lnz_per_site", C.c_double),
        ("trace", C.c_double),
        ("m_imp", C.c_double),
        ("nn_imp", C.c_double),
        ("e_imp", C.c_double),
        ("X", C.c_double),
        ("last_axis", C.c_int),
        ("last_side", C.c_int * 4),
        ("last_k", C.c_int * 4),
        ("last_eps", C.c_double * 4),
        ("min_cut_gap", C.c_double),
        ("flagged", C.c_int),
        ("last_cn", C.c_double),
        ("device_bytes", C.c_size_t),
        ("eig_sweeps", C.c_int),
        ("eig_residual", C.c_double),
        ("block_sparse", C.c_int),
    ]

    def as_dict(self):
        return dict(n=self.n, dims=tuple(self.dims), lnz_per_site=self.lnz_per_site, trace=self.trace,
                    m_imp=self.m_imp, nn_imp=self.nn_imp, e_imp=self.e_imp, X=self.X,
                    last_axis=self.last_axis, last_side=tuple(self.last_side), last_k=tuple(self.last_k),
                    last_eps=tuple(self.last_eps), min_cut_gap=self.min_cut_gap, flagged=self.flagged,
                    last_cn=self.last_cn, device_bytes=self.device_bytes, eig_sweeps=self.eig_sweeps,
                    eig_residual=self.eig_residual, block_sparse=self.block_sparse)


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (no compute); raises HotrgUnavailable if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HotrgUnavailable(f"{path} not built; run python -m paper_1906_06060_amd.build")
    # torch ships its own HIP runtime; initialise it before the library is
    # mapped so both resolve to the same runtime (the device lives there)
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    sig = {
        "hotrg_init": ([C.c_double, C.c_double, C.c_int, C.POINTER(P)], C.c_int),
        "hotrg_init_ex": ([C.c_double, C.c_double, C.c_int, C.POINTER(Config), C.POINTER(P)], C.c_int),
        "hotrg_step": ([P, C.c_int], C.c_int),
        "hotrg_lnZ": ([P, dp], C.c_int),
        "hotrg_observables": ([P, C.POINTER(Obs)], C.c_int),
        "hotrg_backward": ([P, dp, dp], C.c_int),
        "hotrg_free": ([P], None),
        "hotrg_last_error": ([], C.c_char_p),
        "hotrg_get_dims": ([P, ip, ip], C.c_int),
        "hotrg_get_tensor": ([P, C.c_int, dp, C.c_size_t], C.c_int),
        "hotrg_set_state": ([P, ip, dp, dp, dp, C.c_int, C.c_double], C.c_int),
        "hotrg_truncate": ([P, C.c_int], C.c_int),
        "hotrg_step_with_isometries": ([P, C.c_int, C.POINTER(dp), ip], C.c_int),
        "hotrg_get_isometry": ([P, C.c_int, dp, C.c_size_t, ip, ip], C.c_int),
        "hotrg_get_spectrum": ([P, C.c_int, C.c_int, dp, C.c_size_t, ip], C.c_int),
        "hotrg_kernel_stats": ([P, C.c_int, dp, C.POINTER(C.c_longlong), dp], C.c_int),
        "hotrg_reset_stats": ([P], C.c_int),
        "hotrg_observables_noalloc": ([P, P, P, ip, C.c_int, C.c_double, C.c_int, C.c_double, P,
                                       C.POINTER(Obs)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise HotrgError(rc, _lib.hotrg_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _current_stream():
    """torch's current stream (initialising torch's ROCm runtime first, which
    the library relies on to find the device)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return C.c_void_p(0)


class TorchAllocator:
    """Device memory for a context from torch's caching allocator, on the
    context's stream (the library calls alloc / free through ctypes)."""

    def __init__(self, stream_ptr: int, fail_after: int | None = None):
        import torch
        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = int(stream_ptr or 0)
        self.fail_after = fail_after      # tests: NULL from the (fail_after + 1)-th request on
        self.calls = 0
        self.live = {}
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, _ctx):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return None
        try:
            p = self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:
            return None
        self.live[p] = int(nbytes)
        return p

    def _free(self, ptr, _ctx):
        if ptr:
            self.live.pop(ptr, None)
            self.torch.cuda.caching_allocator_delete(ptr)

    @property
    def bytes_held(self) -> int:
        return sum(self.live.values())


_live_contexts = weakref.WeakSet()


@atexit.register
def _close_live_contexts():
    # free every context while the interpreter (and torch) can still serve
    # the allocator callbacks
    for ctx in list(_live_contexts):
        try:
            ctx.close()
        except Exception:
            pass


class Context:
    """One HOTRG coarse-graining state on the GPU (hotrg_ctx).

    allocator="torch" (default when torch sees a GPU): the context's device
    buffers come from torch's caching allocator; "hip": from hipMalloc inside
    the library; or a TorchAllocator instance."""

    def __init__(self, beta: float, h: float, dcut: int, precision: int = FP64, impurities: bool = True,
                 keep_checkpoints: bool = False, mixed_from_step: int = 0, tau_deg: float = 0.0, stream=None,
                 slice_budget: int = 0, eig_max_sweeps: int = 0, mem_budget: int = 0, allocator="torch",
                 dense_only: bool = False):
        lib = load()
        self._h = C.c_void_p()
        stream = stream if stream is not None else _current_stream()
        if allocator == "torch":
            allocator = TorchAllocator(stream.value if isinstance(stream, C.c_void_p) else stream)
        elif allocator == "hip":
            allocator = None
        self.allocator = allocator
        cfg = Config(precision, int(impurities), int(keep_checkpoints), mixed_from_step, tau_deg, stream,
                     slice_budget, eig_max_sweeps)
        if allocator is not None:
            cfg.alloc, cfg.free = allocator.alloc_fn, allocator.free_fn
        cfg.mem_budget = mem_budget
        cfg.dense_only = int(dense_only)
        self.beta, self.h, self.dcut = beta, h, dcut
        self.impurities = impurities
        _check(lib.hotrg_init_ex(beta, h, dcut, C.byref(cfg), C.byref(self._h)))
        _live_contexts.add(self)

    def close(self):
        if self._h:
            _lib.hotrg_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, axis: int):
        _check(_lib.hotrg_step(self._h, axis))

    def truncate(self, axis: int):
        """Environment / eigh / cut stage of a step along `axis` only (state unchanged)."""
        _check(_lib.hotrg_truncate(self._h, axis))

    def step_with_isometries(self, axis: int, Us: dict):
        arrs = [np.ascontiguousarray(Us[q], dtype=np.float64) if q in Us else None for q in range(4)]
        ptrs = (C.POINTER(C.c_double) * 4)(*[_dptr(a) if a is not None else C.POINTER(C.c_double)() for a in arrs])
        ks = (C.c_int * 4)(*[a.shape[1] if a is not None else 0 for a in arrs])
        _check(_lib.hotrg_step_with_isometries(self._h, axis, ptrs, ks))

    def lnz(self) -> float:
        v = C.c_double()
        _check(_lib.hotrg_lnZ(self._h, C.byref(v)))
        return v.value

    def observables(self) -> dict:
        o = Obs()
        _check(_lib.hotrg_observables(self._h, C.byref(o)))
        return o.as_dict()

    def backward(self):
        db, dh = C.c_double(), C.c_double()
        _check(_lib.hotrg_backward(self._h, C.byref(db), C.byref(dh)))
        return db.value, dh.value

    def dims(self):
        d = (C.c_int * 4)()
        n = C.c_int()
        _check(_lib.hotrg_get_dims(self._h, d, C.byref(n)))
        return tuple(d), n.value

    def tensor(self, which: int = 0) -> np.ndarray:
        dims, _ = self.dims()
        shape = []
        for D in dims:
            shape += [D, D]
        out = np.empty(shape, dtype=np.float64)
        _check(_lib.hotrg_get_tensor(self._h, which, _dptr(out), out.size))
        return out

    def set_state(self, T, Sm=None, Se=None, n: int = 0, lnz_acc: float = 0.0):
        T = np.ascontiguousarray(T, dtype=np.float64)
        dims = (C.c_int * 4)(*T.shape[::2])
        Sm = None if Sm is None else np.ascontiguousarray(Sm, dtype=np.float64)
        Se = None if Se is None else np.ascontiguousarray(Se, dtype=np.float64)
        null = C.POINTER(C.c_double)()
        _check(_lib.hotrg_set_state(self._h, dims, _dptr(T), _dptr(Sm) if Sm is not None else null,
                                    _dptr(Se) if Se is not None else null, n, lnz_acc))

    def isometry(self, q: int) -> np.ndarray:
        buf = np.empty(256 * 256)
        r, c = C.c_int(), C.c_int()
        _check(_lib.hotrg_get_isometry(self._h, q, _dptr(buf), buf.size, C.byref(r), C.byref(c)))
        return buf[: r.value * c.value].reshape(r.value, c.value).copy()

    def spectrum(self, q: int, side: int) -> np.ndarray:
        buf = np.empty(256)
        n = C.c_int()
        _check(_lib.hotrg_get_spectrum(self._h, q, side, _dptr(buf), buf.size, C.byref(n)))
        return buf[: n.value].copy()

    def gemm_stats(self):
        ms, fl = C.c_double(), C.c_double()
        ln = C.c_longlong()
        _check(_lib.hotrg_kernel_stats(self._h, 0, C.byref(ms), C.byref(ln), C.byref(fl)))
        return dict(ms=ms.value, launches=ln.value, flops=fl.value)

    def z2_tile_launches(self):
        """Last isometry products since the last reset that wrote their bf16
        Z2 operand blocks through LDS tiles (hotrg_kernel_stats kernel 4)."""
        ln = C.c_longlong()
        _check(_lib.hotrg_kernel_stats(self._h, 4, None, C.byref(ln), None))
        return ln.value

    def z2_reverse_steps(self):
        """Reverse-pass steps since the last reset undone in the Z2 block form
        (hotrg_kernel_stats kernel 5)."""
        ln = C.c_longlong()
        _check(_lib.hotrg_kernel_stats(self._h, 5, None, C.byref(ln), None))
        return ln.value

    def phase_stats(self):
        """Device ms per phase of hotrg_step since the last reset (kernels 1..3),
        the GEMM ms (kernel 0) and the number of steps counted."""
        out = {}
        for kern, name in ((1, "isometries_ms"), (2, "contraction_ms"), (3, "normalise_ms"), (0, "gemm_ms")):
            ms, fl = C.c_double(), C.c_double()
            ln = C.c_longlong()
            _check(_lib.hotrg_kernel_stats(self._h, kern, C.byref(ms), C.byref(ln), C.byref(fl)))
            out[name] = ms.value
            if kern == 1:
                out["steps"] = ln.value
        return out

    def reset_stats(self):
        _check(_lib.hotrg_reset_stats(self._h))


def observables_noalloc(T_ptr: int, dims, axis: int, h: float = 0.0, n: int = 0, lnz_acc: float = 0.0,
                        Sm_ptr: int = 0, Se_ptr: int = 0, stream=None) -> dict:
    """hotrg_observables_noalloc on caller-held device tensors (raw device
    pointers, e.g. torch tensors' data_ptr()); allocates nothing on the device."""
    lib = load()
    o = Obs()
    d = (C.c_int * 4)(*dims)
    st = stream if stream is not None else _current_stream()
    _check(lib.hotrg_observables_noalloc(C.c_void_p(T_ptr), C.c_void_p(Sm_ptr or None), C.c_void_p(Se_ptr or None),
                                         d, axis, h, n, lnz_acc, st, C.byref(o)))
    return o.as_dict()


def flow(beta: float, h: float, dcut: int, nsteps: int, axes=None, **kw):
    """Run nsteps steps (axes cycling x, y, z, t) and return per-step observables."""
    out = []
    with Context(beta, h, dcut, **kw) as ctx:
        for n in range(nsteps):
            ctx.step(axes[n] if axes is not None else n % 4)
            out.append(ctx.observables())
    return out
