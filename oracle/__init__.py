"""FP64 CPU oracle of the lattice Boltzmann step for the Bona-Masso system.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package.  It is a plain, slow,
scalar C implementation (``lbref.c``) written from the paper, sharing no code
with the GPU library; this module only marshals arguments through ctypes.

Arrays: u is float64 (16, nz, ny, nx); f is float64 (16, Q, nz, ny, nx),
the distributions at the current time (after streaming), Q = 19 on D3Q19 and
Q = 9 on D2Q9 (which takes nz = 1).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build

HARMONIC = 0
GEODESIC = 1
ONE_PLUS_LOG = 2
D3Q19 = 19
D2Q9 = 9
MATTER_TENSOR = 0
MATTER_FLUID = 1
COLLISION_BGK = 0
COLLISION_REGULARIZED = 1
NF = 16
NQ = 19

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.lbref_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_int, ctypes.POINTER(P)]
    lib.lbref_create.restype = ctypes.c_int
    lib.lbref_create_lattice.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_int, ctypes.POINTER(P)]
    lib.lbref_create_lattice.restype = ctypes.c_int
    lib.lbref_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
    lib.lbref_lattice.restype = ctypes.c_int
    lib.lbref_destroy.argtypes = [P]
    lib.lbref_destroy.restype = None
    lib.lbref_init_fields.argtypes = [P, dp]
    lib.lbref_step.argtypes = [P, ctypes.c_longlong]
    lib.lbref_moments.argtypes = [P, dp]
    lib.lbref_get_distributions.argtypes = [P, dp]
    lib.lbref_set_distributions.argtypes = [P, dp]
    lib.lbref_nsteps_done.argtypes = [P]
    lib.lbref_nsteps_done.restype = ctypes.c_longlong
    lib.lbref_lattice_d3q19.argtypes = [ctypes.POINTER(ctypes.c_int), dp]
    lib.lbref_lattice_d3q19.restype = None
    lib.lbref_point_rhs.argtypes = [dp, ctypes.c_int, dp]
    lib.lbref_point_rhs_matter.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, dp]
    lib.lbref_set_matter.argtypes = [P, ctypes.c_int, dp, ctypes.c_int]
    lib.lbref_set_collision.argtypes = [P, ctypes.c_int]
    lib.lbref_point_feq.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
    lib.lbref_point_feq.restype = None
    lib.lbref_num_threads.argtypes = []
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


class Oracle:
    """One periodic lattice evolved by the CPU oracle."""

    def __init__(self, nx: int, ny: int, nz: int, tau: float, slicing: int = HARMONIC, lattice: int = D3Q19,
                 collision: int = COLLISION_BGK):
        lib = _load()
        self._lib = lib
        self.shape = (nz, ny, nx)
        self.nsite = nx * ny * nz
        self.nq = int(lattice)
        h = ctypes.c_void_p()
        _check(lib.lbref_create_lattice(int(lattice), nx, ny, nz, float(tau), int(slicing), ctypes.byref(h)),
               "create")
        self._h = h
        _check(lib.lbref_set_collision(h, int(collision)), "set_collision")

    def close(self) -> None:
        if self._h:
            self._lib.lbref_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, u0: np.ndarray) -> None:
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        assert u0.shape == (NF,) + self.shape, u0.shape
        _check(self._lib.lbref_init_fields(self._h, _dp(u0)), "init_fields")

    def step(self, n: int = 1) -> None:
        _check(self._lib.lbref_step(self._h, int(n)), "step")

    def moments(self) -> np.ndarray:
        out = np.empty((NF,) + self.shape, dtype=np.float64)
        _check(self._lib.lbref_moments(self._h, _dp(out)), "moments")
        return out

    def distributions(self) -> np.ndarray:
        out = np.empty((NF, self.nq) + self.shape, dtype=np.float64)
        _check(self._lib.lbref_get_distributions(self._h, _dp(out)), "get_distributions")
        return out

    def set_distributions(self, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (NF, self.nq) + self.shape
        _check(self._lib.lbref_set_distributions(self._h, _dp(f)), "set_distributions")

    def set_matter(self, M, kind: int = MATTER_TENSOR) -> None:
        """Matter in lattice units: kind MATTER_TENSOR, M = G^00, G^0_k, G_ij
        (10 values); kind MATTER_FLUID, M = (rho, P).  M of shape (ncomp,)
        applies at every site, (ncomp, nz, ny, nx) per site; None: vacuum."""
        if M is None:
            _check(self._lib.lbref_set_matter(self._h, int(kind), None, 0), "set_matter")
            return
        nc = 2 if kind == MATTER_FLUID else 10
        M = np.ascontiguousarray(M, dtype=np.float64)
        if M.shape == (nc,):
            _check(self._lib.lbref_set_matter(self._h, int(kind), _dp(M), 0), "set_matter")
        else:
            assert M.shape == (nc,) + self.shape, M.shape
            _check(self._lib.lbref_set_matter(self._h, int(kind), _dp(M), 1), "set_matter")

    @property
    def steps_done(self) -> int:
        return int(self._lib.lbref_nsteps_done(self._h))


def lattice_d3q19():
    lib = _load()
    c = (ctypes.c_int * 57)()
    w = np.empty(19, dtype=np.float64)
    lib.lbref_lattice_d3q19(c, _dp(w))
    return np.array(list(c), dtype=np.int64).reshape(19, 3), w


def lattice(q: int):
    """Velocities (Q, 3) and weights (Q,) of the oracle's D3Q19 or D2Q9 table."""
    lib = _load()
    c = (ctypes.c_int * (3 * q))()
    w = np.empty(q, dtype=np.float64)
    _check(0 if lib.lbref_lattice(int(q), c, _dp(w)) == q else -1, "lattice")
    return np.array(list(c), dtype=np.int64).reshape(q, 3), w


def point_rhs(alpha, g6, K6, V, A, D18, slicing: int = HARMONIC, matter=None, kind: int = MATTER_TENSOR) -> dict:
    """Right-hand sides and flux of the Bona-Masso system at one point;
    matter: None (vacuum), G^00, G^0_k, G_ij (10 values, kind MATTER_TENSOR)
    or (rho, P) (kind MATTER_FLUID)."""
    lib = _load()
    inp = np.concatenate([[alpha], g6, K6, V, A, D18]).astype(np.float64)
    assert inp.shape == (37,)
    out = np.empty(34, dtype=np.float64)
    if matter is None:
        _check(lib.lbref_point_rhs(_dp(inp), int(slicing), _dp(out)), "point_rhs")
    else:
        G = np.ascontiguousarray(matter, dtype=np.float64)
        assert G.shape == ((2,) if kind == MATTER_FLUID else (10,))
        _check(lib.lbref_point_rhs_matter(_dp(inp), int(kind), _dp(G), int(slicing), _dp(out)), "point_rhs")
    return {
        "R_alpha": out[0],
        "R_gamma": out[1:7].copy(),
        "R_K": out[7:13].copy(),
        "Omega": out[13:16].copy(),
        "lambda": out[16:34].reshape(3, 6).copy(),
    }


def point_feq(kind: int, u: float, F=(0.0, 0.0, 0.0)) -> np.ndarray:
    lib = _load()
    Fa = np.asarray(F, dtype=np.float64)
    out = np.empty(19, dtype=np.float64)
    lib.lbref_point_feq(int(kind), float(u), _dp(Fa), _dp(out))
    return out


def num_threads() -> int:
    return int(_load().lbref_num_threads())
