"""Closed-form initial data for the wave tests (paper, section "Tests and Results").

Lattice units throughout: site i sits at coordinate x = i and step n at time
t = n (dt = dx = 1).  The vacuum equations are scale free, so a physical run
with wavelength d_phys and spacing dx equals a lattice run with d = d_phys/dx.

Gauge wave (section "Gauge Wave"): ds^2 = -H dt^2 + H dx^2 + dy^2 + dz^2 with
H = 1 - A sin(2 pi (x - t)/d).  Then alpha = sqrt(H), gamma_xx = H and the only
non-zero curvature component is K_xx = -(pi A/d) cos(2 pi (x - t)/d)/sqrt(H).
The same metric written along a unit direction n (a spatial rotation of the
coordinates) reads gamma_ij = delta_ij + (H - 1) n_i n_j and
K_ij = -(pi A/d) cos(phi)/sqrt(H) n_i n_j with phi = 2 pi (n.x - t)/d.
For both, V_k (section "Bona-Masso formulation", its definition from D) is 0.

Linear wave (section "Linear Wave"): gamma_yy = 1 + b, gamma_zz = 1 - b,
b = A sin(2 pi (x - t)/d), alpha = 1, K_yy = -K_zz = (pi A/d) cos(...).
V_x follows from its definition V_k = D_kr^r - D^r_rk with D = (1/2) d gamma.
"""

from __future__ import annotations

import math

import numpy as np

NFIELDS = 16
FIELD_NAMES = (
    "alpha",
    "gxx", "gxy", "gxz", "gyy", "gyz", "gzz",
    "Kxx", "Kxy", "Kxz", "Kyy", "Kyz", "Kzz",
    "Vx", "Vy", "Vz",
)
# symmetric storage order of a 3x3 tensor: (xx, xy, xz, yy, yz, zz)
SYM_PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def _grid(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(
        np.arange(nz, dtype=np.float64),
        np.arange(ny, dtype=np.float64),
        np.arange(nx, dtype=np.float64),
        indexing="ij",
    )
    return x, y, z


def minkowski(nx: int, ny: int, nz: int) -> np.ndarray:
    """Flat space at rest: alpha = 1, gamma = delta, K = V = 0."""
    u = np.zeros((NFIELDS, nz, ny, nx), dtype=np.float64)
    u[0] = 1.0
    u[1] = 1.0
    u[4] = 1.0
    u[6] = 1.0
    return u


def _fill_wave(u: np.ndarray, H: np.ndarray, kfac: np.ndarray, n) -> None:
    """alpha = sqrt(H), gamma = delta + (H-1) n n, K = kfac n n."""
    u[0] = np.sqrt(H)
    for s, (i, j) in enumerate(SYM_PAIRS):
        nn = n[i] * n[j]
        u[1 + s] = (1.0 if i == j else 0.0) + (H - 1.0) * nn
        u[7 + s] = kfac * nn
    u[13:16] = 0.0


def gauge_wave_x(nx: int, ny: int, nz: int, A: float, d: float, t: float = 0.0) -> np.ndarray:
    """Gauge wave travelling along +x at time t (paper, section "Gauge Wave")."""
    x, _, _ = _grid(nx, ny, nz)
    phi = 2.0 * math.pi * (x - t) / d
    H = 1.0 - A * np.sin(phi)
    kfac = -(math.pi * A / d) * np.cos(phi) / np.sqrt(H)
    u = np.zeros((NFIELDS, nz, ny, nx), dtype=np.float64)
    _fill_wave(u, H, kfac, (1.0, 0.0, 0.0))
    return u


def gauge_wave_diag(n: int, nz: int, A: float, t: float = 0.0) -> np.ndarray:
    """Gauge wave along (1,1,0)/sqrt(2) on an n x n x nz periodic lattice.

    The wavelength is d = n/sqrt(2), so the phase 2 pi (x + y - sqrt(2) t)/n is
    periodic with period n along both x and y.  One crossing takes d steps.
    """
    x, y, _ = _grid(n, n, nz)
    phi = 2.0 * math.pi * (x + y - math.sqrt(2.0) * t) / n
    d = n / math.sqrt(2.0)
    H = 1.0 - A * np.sin(phi)
    kfac = -(math.pi * A / d) * np.cos(phi) / np.sqrt(H)
    u = np.zeros((NFIELDS, nz, n, n), dtype=np.float64)
    r = 1.0 / math.sqrt(2.0)
    _fill_wave(u, H, kfac, (r, r, 0.0))
    return u


def gauge_wave_dir(nx, ny, nz, direction, A, d, t=0.0, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Gauge wave along an arbitrary direction (not lattice periodic in general)."""
    nvec = np.asarray(direction, dtype=np.float64)
    nvec = nvec / np.linalg.norm(nvec)
    x, y, z = _grid(nx, ny, nz)
    s = nvec[0] * (x + origin[0]) + nvec[1] * (y + origin[1]) + nvec[2] * (z + origin[2])
    phi = 2.0 * math.pi * (s - t) / d
    H = 1.0 - A * np.sin(phi)
    kfac = -(math.pi * A / d) * np.cos(phi) / np.sqrt(H)
    u = np.zeros((NFIELDS, nz, ny, nx), dtype=np.float64)
    _fill_wave(u, H, kfac, tuple(nvec))
    return u


def linear_wave_x(nx: int, ny: int, nz: int, A: float, d: float, t: float = 0.0) -> np.ndarray:
    """Linearised gravitational wave along x (paper, section "Linear Wave")."""
    x, _, _ = _grid(nx, ny, nz)
    phi = 2.0 * math.pi * (x - t) / d
    b = A * np.sin(phi)
    bx = A * (2.0 * math.pi / d) * np.cos(phi)
    u = minkowski(nx, ny, nz)
    u[4] = 1.0 + b
    u[6] = 1.0 - b
    u[10] = (math.pi * A / d) * np.cos(phi)
    u[12] = -(math.pi * A / d) * np.cos(phi)
    # V_x = gamma^yy D_xyy + gamma^zz D_xzz (the D^r_rx part vanishes)
    u[13] = 0.5 * bx / (1.0 + b) - 0.5 * bx / (1.0 - b)
    return u


def add_lapse_noise(u: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """Add iid Gaussian noise of standard deviation sigma to the lapse (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = u.copy()
    out[0] += sigma * rng.standard_normal(out[0].shape)
    return out


def random_state(nx: int, ny: int, nz: int, seed: int, amp: float = 0.05) -> np.ndarray:
    """Seeded random perturbation of flat space in every field.

    gamma stays symmetric positive definite for amp < 0.3; alpha stays near 1.
    Used for element-wise parity runs where any state is a valid input.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = minkowski(nx, ny, nz)
    u += amp * rng.uniform(-1.0, 1.0, size=u.shape)
    return u


def random_matter(nx: int, ny: int, nz: int, seed: int, amp: float = 1e-3, ncomp: int = 10) -> np.ndarray:
    """Seeded random matter values per site, shape (ncomp, nz, ny, nx):
    U(-amp, amp) in every component (10 for a tensor G^00, G^0_k, G_ij;
    2 for a fluid's rho, P, which are drawn in U(0, amp))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if ncomp == 2:
        return amp * rng.uniform(0.0, 1.0, size=(2, nz, ny, nx))
    return amp * rng.uniform(-1.0, 1.0, size=(ncomp, nz, ny, nx))


def crossing_steps_x(d: float) -> float:
    """Steps for one crossing of a wave of wavelength d (light speed 1)."""
    return float(d)


def crossing_steps_diag(n: int) -> float:
    """Steps for one crossing of the (1,1,0) wave on an n x n lattice."""
    return n / math.sqrt(2.0)
