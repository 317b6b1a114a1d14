"""Flat FLRW universe with a perfect fluid P = w rho (section "Expansion of
flat universe"; the paper's case is w = 1, P = rho = 1/(3 t^2)).

Comoving coordinates, alpha = 1, gamma_ij = a(t)^2 delta_ij with
a = t^q, q = 2 / (3 (1 + w)) (units c = 8 pi G = 1, so rho = 3 (a'/a)^2), and
K_ij = -d_t gamma_ij / 2 = -q t^(2q - 1) delta_ij.

Lattice units: a run with physical time step dt maps t = t0 + n dt to step n;
lengths scale by 1/dt, so K (1/length) carries a factor dt and rho, P
(1/length^2) carry dt^2.  Closed forms only; no part of the scheme.
"""

from __future__ import annotations

import numpy as np


def _q(w: float) -> float:
    return 2.0 / (3.0 * (1.0 + w))


def flrw_exact(t: float, w: float = 1.0):
    """(gamma_xx, K_xx, rho, P) of the exact solution at physical time t."""
    q = _q(w)
    rho = 3.0 * (q / t) ** 2
    return t ** (2.0 * q), -q * t ** (2.0 * q - 1.0), rho, w * rho


def flrw_fields(nx: int, ny: int, nz: int, dt: float, t0: float = 1.0, w: float = 1.0) -> np.ndarray:
    """Fields (16, nz, ny, nx) at t0 in lattice units."""
    g, k, _, _ = flrw_exact(t0, w)
    u = np.zeros((16, nz, ny, nx))
    u[0] = 1.0
    for p in (0, 3, 5):
        u[1 + p] = g
        u[7 + p] = k * dt
    return u


def flrw_fluid(t: float, dt: float, w: float = 1.0) -> np.ndarray:
    """(rho, P) of the fluid at physical time t, in lattice units."""
    _, _, rho, P = flrw_exact(t, w)
    return np.array([rho * dt * dt, P * dt * dt])
