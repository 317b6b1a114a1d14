"""Thin ctypes binding of the C-ABI in include/lb.h.

Argument marshalling only: every step of the lattice Boltzmann path runs in
the HIP library (liblbnr.so).  There is no CPU fallback; if the library is
missing this module raises on import of the first handle.

Arrays: host arrays are numpy float64 C-contiguous; device arrays are torch
float64 CUDA tensors (their data pointer is passed with on_device = 1 and the
call is ordered on the handle's stream).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbnr.so")

LB_OK = 0
LB_EINVAL = -1
LB_ENOMEM = -2
LB_EDEVICE = -3
LB_ESTATE = -4
LB_D3Q19 = 19
LB_D2Q9 = 9
D3Q19 = LB_D3Q19
D2Q9 = LB_D2Q9
HARMONIC = 0
GEODESIC = 1
ONE_PLUS_LOG = 2
FP64 = 0
FP32_DEV = 1
PATH_AUTO = 0
PATH_SPLIT = 1
PATH_FUSED = 2
MATTER_TENSOR = 0
MATTER_FLUID = 1
COLLISION_BGK = 0
COLLISION_REGULARIZED = 1
NF = 16
NQ = 19

EXPORTS = (
    "lb_create", "lb_device_bytes", "lb_init_fields", "lb_step", "lb_moments",
    "lb_get_distributions", "lb_error_norms", "lb_steps_done", "lb_set_timing",
    "lb_kernel_times", "lb_set_matter", "lb_set_distributions", "lb_check_finite", "lb_destroy",
    "lb_strerror", "lb_last_error",
)


# lb_dev_alloc_fn / lb_dev_free_fn of include/lb.h
DEV_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DEV_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class LBConfig(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("slicing", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("path", ctypes.c_int),
        ("collision", ctypes.c_int),
        ("dev_alloc", DEV_ALLOC_FN),
        ("dev_free", DEV_FREE_FN),
        ("alloc_ctx", ctypes.c_void_p),
    ]


class LBError(RuntimeError):
    pass


_lib = None


def load_library():
    """Load liblbnr.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LBError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.lb_create.argtypes = [ctypes.POINTER(LBConfig), PP]
    lib.lb_device_bytes.argtypes = [ctypes.POINTER(LBConfig)]
    lib.lb_device_bytes.restype = ctypes.c_size_t
    lib.lb_init_fields.argtypes = [P, P, ctypes.c_int]
    lib.lb_step.argtypes = [P, ctypes.c_longlong]
    lib.lb_moments.argtypes = [P, P, ctypes.c_int]
    lib.lb_get_distributions.argtypes = [P, P, ctypes.c_int]
    lib.lb_error_norms.argtypes = [P, P, ctypes.c_int, dp, dp, dp]
    lib.lb_steps_done.argtypes = [P]
    lib.lb_steps_done.restype = ctypes.c_longlong
    lib.lb_set_timing.argtypes = [P, ctypes.c_int]
    lib.lb_kernel_times.argtypes = [P, ctypes.POINTER(ctypes.c_char_p), dp, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int)]
    lib.lb_set_matter.argtypes = [P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int]
    lib.lb_set_distributions.argtypes = [P, P, ctypes.c_int]
    lib.lb_check_finite.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
    lib.lb_destroy.argtypes = [P]
    lib.lb_destroy.restype = None
    lib.lb_strerror.argtypes = [ctypes.c_int]
    lib.lb_strerror.restype = ctypes.c_char_p
    lib.lb_last_error.argtypes = []
    lib.lb_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != LB_OK:
        lib = load_library()
        msg = lib.lb_strerror(rc).decode()
        extra = lib.lb_last_error().decode()
        raise LBError(f"{what}: {msg} ({rc}) {extra}".rstrip())


def _ptr(a, nelem: int):
    """(pointer, on_device) of a numpy array or a torch tensor of nelem doubles."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags.c_contiguous or a.size != nelem:
            raise ValueError("expected a C-contiguous float64 array of %d elements" % nelem)
        return ctypes.c_void_p(a.ctypes.data), 0
    import torch  # device arrays are torch tensors

    if not isinstance(a, torch.Tensor):
        raise TypeError("expected numpy array or torch tensor")
    if a.dtype != torch.float64 or not a.is_contiguous() or a.numel() != nelem:
        raise ValueError("expected a contiguous float64 tensor of %d elements" % nelem)
    if a.is_cuda:
        # The library reads and writes device arrays on the handle's stream,
        # which does not wait for torch's: let torch's pending work on this
        # tensor finish first.
        torch.cuda.current_stream(a.device).synchronize()
        return ctypes.c_void_p(a.data_ptr()), 1
    return ctypes.c_void_p(a.data_ptr()), 0


def make_config(nx, ny, nz, tau, slicing=HARMONIC, precision=FP64, device=-1, stream=None,
                path=PATH_AUTO, lattice=LB_D3Q19, collision=COLLISION_BGK, hooks=None) -> LBConfig:
    """hooks: None, or a (DEV_ALLOC_FN, DEV_FREE_FN) pair the caller keeps alive."""
    cfg = LBConfig(int(lattice), int(nx), int(ny), int(nz), float(tau), int(slicing), int(precision),
                   int(device), ctypes.c_void_p(stream) if stream else None, int(path), int(collision))
    if hooks is not None:
        cfg.dev_alloc, cfg.dev_free = hooks
    return cfg


class DeviceAllocator:
    """A device allocator for the library (the dev_alloc/dev_free hooks):
    alloc(nbytes) returns a device address (int) or None, free(ptr) gives it
    back.  hooks() wraps them as C callbacks, which must stay alive as long as
    the handle (Lattice keeps them)."""

    def alloc(self, nbytes: int):
        raise NotImplementedError

    def free(self, ptr: int) -> None:
        raise NotImplementedError

    def hooks(self):
        def _alloc(nbytes, _ctx):
            try:
                p = self.alloc(int(nbytes))
            except Exception:  # an exception cannot cross the C boundary: report no memory
                return None
            return int(p) if p else None

        def _free(ptr, _ctx):
            try:
                self.free(int(ptr))
            except Exception:
                pass

        return DEV_ALLOC_FN(_alloc), DEV_FREE_FN(_free)


class TorchAllocator(DeviceAllocator):
    """Serves the library from torch's caching allocator on `device`, so its
    buffers count in torch.cuda.memory_allocated() and come from (and go back
    to) torch's pool."""

    def __init__(self, device: int = 0):
        self.device = int(device)

    def alloc(self, nbytes: int):
        import torch

        return torch.cuda.caching_allocator_alloc(nbytes, device=self.device)

    def free(self, ptr: int) -> None:
        import torch

        torch.cuda.caching_allocator_delete(ptr)


def device_bytes(nx, ny, nz, tau=0.6, precision=FP64, lattice=LB_D3Q19, path=PATH_AUTO) -> int:
    cfg = make_config(nx, ny, nz, tau, precision=precision, lattice=lattice, path=path)
    return int(load_library().lb_device_bytes(ctypes.byref(cfg)))


class Lattice:
    """One periodic lattice evolved on the GPU (lb_create ... lb_destroy)."""

    def __init__(self, nx: int, ny: int, nz: int, tau: float, slicing: int = HARMONIC,
                 precision: int = FP64, device: int = -1, stream=None, path: int = PATH_AUTO,
                 lattice: int = LB_D3Q19, collision: int = COLLISION_BGK, allocator=None):
        """allocator: None (the library's hipMalloc), "torch" (torch's caching
        allocator on `device`) or a DeviceAllocator."""
        lib = load_library()
        self._lib = lib
        self.shape = (nz, ny, nx)
        self.nsite = nx * ny * nz
        self.nq = int(lattice)
        if allocator == "torch":
            allocator = TorchAllocator(device if device >= 0 else 0)
        self._hooks = allocator.hooks() if allocator is not None else None  # alive until lb_destroy
        cfg = make_config(nx, ny, nz, tau, slicing, precision, device, stream, path, lattice, collision,
                          hooks=self._hooks)
        h = ctypes.c_void_p()
        _check(lib.lb_create(ctypes.byref(cfg), ctypes.byref(h)), "lb_create")
        self._h = h

    def close(self) -> None:
        if self._h:
            self._lib.lb_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, u0) -> None:
        p, dev = _ptr(u0, NF * self.nsite)
        _check(self._lib.lb_init_fields(self._h, p, dev), "lb_init_fields")

    def step(self, n: int = 1) -> None:
        _check(self._lib.lb_step(self._h, int(n)), "lb_step")

    def moments(self, out=None):
        if out is None:
            out = np.empty((NF,) + self.shape, dtype=np.float64)
        p, dev = _ptr(out, NF * self.nsite)
        _check(self._lib.lb_moments(self._h, p, dev), "lb_moments")
        return out

    def distributions(self, out=None):
        if out is None:
            out = np.empty((NF, self.nq) + self.shape, dtype=np.float64)
        p, dev = _ptr(out, NF * self.nq * self.nsite)
        _check(self._lib.lb_get_distributions(self._h, p, dev), "lb_get_distributions")
        return out

    def set_distributions(self, f) -> None:
        """Restore a state saved with distributions() (checkpoint/resume)."""
        p, dev = _ptr(f, NF * self.nq * self.nsite)
        _check(self._lib.lb_set_distributions(self._h, p, dev), "lb_set_distributions")

    def check_finite(self) -> bool:
        """True if every moment of every site is finite."""
        ok = ctypes.c_int()
        _check(self._lib.lb_check_finite(self._h, ctypes.byref(ok)), "lb_check_finite")
        return bool(ok.value)

    def set_matter(self, M, kind: int = MATTER_TENSOR) -> None:
        """Matter in lattice units (lb_set_matter): kind MATTER_TENSOR, M =
        G^00, G^0_k, G_ij; kind MATTER_FLUID, M = (rho, P).  M with one value
        per component applies at every site; (ncomp, nz, ny, nx) per site;
        None returns to vacuum."""
        if M is None:
            _check(self._lib.lb_set_matter(self._h, int(kind), None, 0, 0), "lb_set_matter")
            return
        nc = 2 if kind == MATTER_FLUID else 10
        if isinstance(M, (list, tuple)):
            M = np.asarray(M, dtype=np.float64)
        per_site = int(M.shape != (nc,))
        p, dev = _ptr(M, nc * (self.nsite if per_site else 1))
        _check(self._lib.lb_set_matter(self._h, int(kind), p, per_site, dev), "lb_set_matter")

    def error_norms(self, u_ref) -> dict:
        p, dev = _ptr(u_ref, NF * self.nsite)
        mx = (ctypes.c_double * NF)()
        l2 = (ctypes.c_double * NF)()
        rm = (ctypes.c_double * NF)()
        _check(self._lib.lb_error_norms(self._h, p, dev, mx, l2, rm), "lb_error_norms")
        return {"max_abs": np.array(mx[:]), "l2": np.array(l2[:]), "ref_max": np.array(rm[:])}

    @property
    def steps_done(self) -> int:
        return int(self._lib.lb_steps_done(self._h))

    def set_timing(self, enable: bool) -> None:
        _check(self._lib.lb_set_timing(self._h, int(bool(enable))), "lb_set_timing")

    def kernel_times(self) -> dict:
        names = (ctypes.c_char_p * 8)()
        ms = (ctypes.c_double * 8)()
        n = ctypes.c_int()
        _check(self._lib.lb_kernel_times(self._h, names, ms, 8, ctypes.byref(n)), "lb_kernel_times")
        return {names[i].decode(): ms[i] for i in range(n.value)}
