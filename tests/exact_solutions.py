"""Exact vacuum solutions of the Einstein equations in zero-shift form.

Used to pin the oracle's Bona-Masso right-hand sides: for an exact solution,
evaluated with analytic derivatives, the evolution equations (sections
"Bona-Masso evolution equations" and "Gauge choices") must hold point-wise:

    d_t alpha  = R_alpha                  (when the slicing condition holds)
    d_t gamma  = R_gamma = -2 alpha K
    d_t K_ij + d_k (alpha lambda^k_ij) = alpha S_ij
    d_t V_k    = Omega_k

Each solution supplies lapse alpha(t, x) and 3-metric gamma_ij(t, x) as sympy
expressions in coordinates (t, x1, x2, x3); K, A, D and V follow from their
definitions (K_ij = -d_t gamma_ij / (2 alpha) for zero shift, A_k = d_k ln alpha,
D_kij = d_k gamma_ij / 2, V_k = D_kr^r - D^r_rk).  Nothing here implements the
lattice Boltzmann scheme or the paper's S_ij / Omega_k / lambda formulas.
"""

from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import numpy as np
import sympy as sp

t, x1, x2, x3 = sp.symbols("t x1 x2 x3", real=True)
X = (x1, x2, x3)
PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


@dataclass
class Solution:
    name: str
    alpha: sp.Expr
    gamma: sp.Matrix           # 3x3 symmetric
    gamma_inv: sp.Matrix       # its inverse (supplied to avoid a symbolic inversion)
    slicing: str | None        # "harmonic", "geodesic" or None (lapse given, not a slicing of ours)
    points: tuple              # evaluation points (t, x1, x2, x3)


def _state_exprs(sol: Solution):
    a, g, gi = sol.alpha, sol.gamma, sol.gamma_inv
    K = -sp.diff(g, t) / (2 * a)
    A = [sp.diff(a, X[k]) / a for k in range(3)]
    D = [[[sp.diff(g[i, j], X[k]) / 2 for j in range(3)] for i in range(3)] for k in range(3)]
    V = []
    for k in range(3):
        v = 0
        for r in range(3):
            for s in range(3):
                v += gi[r, s] * D[k][r][s] - gi[r, s] * D[s][r][k]
        V.append(v)
    return a, g, K, V, A, D


@functools.lru_cache(maxsize=None)
def compiled(name: str):
    """Lambdified state and exact time derivatives of a named solution."""
    sol = SOLUTIONS[name]()
    a, g, K, V, A, D = _state_exprs(sol)
    state = [a] + [g[i, j] for i, j in PAIRS] + [K[i, j] for i, j in PAIRS] + list(V) + list(A) \
        + [D[k][i][j] for k in range(3) for i, j in PAIRS]
    dt = [sp.diff(a, t)] + [sp.diff(g[i, j], t) for i, j in PAIRS] \
        + [sp.diff(K[i, j], t) for i, j in PAIRS] + [sp.diff(v, t) for v in V]
    fs = sp.lambdify((t, x1, x2, x3), state, modules="mpmath", cse=True)
    fd = sp.lambdify((t, x1, x2, x3), dt, modules="mpmath", cse=True)
    return sol, fs, fd


def evaluate(name: str, point):
    """(state[37], dt[16]) as float64 at point = (t, x1, x2, x3)."""
    import mpmath

    _, fs, fd = compiled(name)
    with mpmath.workdps(40):
        s = [float(sp.re(v)) if isinstance(v, complex) else float(mpmath.re(v)) for v in fs(*point)]
        d = [float(mpmath.re(v)) for v in fd(*point)]
    return np.array(s), np.array(d)


# --------------------------------------------------------------------------
# the solutions
# --------------------------------------------------------------------------

def _unit(v):
    n = math.sqrt(sum(c * c for c in v))
    return [sp.Rational(c) / sp.sqrt(sum(c * c for c in v)) for c in v], n


def gauge_wave_general() -> Solution:
    """Gauge wave along (1, 2, 3)/sqrt(14): Minkowski in moving coordinates,
    harmonic slicing (section "Gauge Wave", rotated)."""
    n, _ = _unit((1, 2, 3))
    Aw, d = sp.Rational(1, 10), sp.Rational(7, 2)
    s = sum(n[i] * X[i] for i in range(3))
    H = 1 - Aw * sp.sin(2 * sp.pi * (s - t) / d)
    g = sp.eye(3) + (H - 1) * sp.Matrix(3, 1, n) * sp.Matrix(1, 3, n)
    gi = sp.eye(3) + (1 / H - 1) * sp.Matrix(3, 1, n) * sp.Matrix(1, 3, n)
    return Solution("gauge_wave_general", sp.sqrt(H), g, gi, "harmonic",
                    ((0.3, 0.1, 0.7, -0.4), (1.1, -0.6, 0.2, 0.9), (2.0, 0.0, 0.0, 0.0)))


def two_gauge_waves() -> Solution:
    """Left- and right-moving gauge waves together: with T - X = F(t - x) and
    T + X = G(t + x), Minkowski becomes F'(t-x) G'(t+x) (-dt^2 + dx^2) + dy^2
    + dz^2.  The time function is a sum of a left and a right mover, so the
    slicing is harmonic.  Rotated to a general direction."""
    n, _ = _unit((2, -1, 1))
    s = sum(n[i] * X[i] for i in range(3))
    H = (1 - sp.Rational(1, 8) * sp.sin(2 * sp.pi * (s - t) / 3)) * \
        (1 - sp.Rational(1, 12) * sp.cos(2 * sp.pi * (s + t) / 5))
    g = sp.eye(3) + (H - 1) * sp.Matrix(3, 1, n) * sp.Matrix(1, 3, n)
    gi = sp.eye(3) + (1 / H - 1) * sp.Matrix(3, 1, n) * sp.Matrix(1, 3, n)
    return Solution("two_gauge_waves", sp.sqrt(H), g, gi, "harmonic",
                    ((0.25, 0.3, -0.2, 0.5), (1.7, 1.0, 0.4, -0.8)))


def _sheared(gdiag, gdiag_inv, M):
    """Metric in coordinates x = M x' (constant M): gamma' = M^T gamma M."""
    Mi = M.inv()
    g = M.T * gdiag * M
    gi = Mi * gdiag_inv * Mi.T
    return g, gi


_SHEAR = sp.Matrix([[1, sp.Rational(1, 5), sp.Rational(-1, 7)],
                    [sp.Rational(1, 9), 1, sp.Rational(1, 4)],
                    [sp.Rational(-1, 6), sp.Rational(1, 3), 1]])


def schwarzschild_isotropic_sheared() -> Solution:
    """Static Schwarzschild in isotropic coordinates, alpha = (1 - M/2r)/(1 + M/2r),
    gamma = psi^4 delta with psi = 1 + M/2r, then a constant linear change of the
    spatial coordinates so that every metric component is non-zero.  K = 0."""
    M = sp.Rational(1, 2)
    y = _SHEAR * sp.Matrix(X)
    r = sp.sqrt(y[0] ** 2 + y[1] ** 2 + y[2] ** 2)
    psi = 1 + M / (2 * r)
    a = (1 - M / (2 * r)) / (1 + M / (2 * r))
    g, gi = _sheared(psi ** 4 * sp.eye(3), psi ** -4 * sp.eye(3), _SHEAR)
    return Solution("schwarzschild_isotropic_sheared", a, g, gi, "geodesic",
                    ((0.0, 1.3, -0.7, 0.9), (0.0, -2.0, 1.1, 0.4)))


def kasner_sheared() -> Solution:
    """Kasner: alpha = 1, gamma = diag(t^2p1, t^2p2, t^2p3) with p = (-1/3, 2/3,
    2/3) (sum p = sum p^2 = 1), sheared by a constant linear map.  D = 0."""
    p = (sp.Rational(-1, 3), sp.Rational(2, 3), sp.Rational(2, 3))
    gd = sp.diag(*[t ** (2 * pk) for pk in p])
    gdi = sp.diag(*[t ** (-2 * pk) for pk in p])
    g, gi = _sheared(gd, gdi, _SHEAR)
    return Solution("kasner_sheared", sp.Integer(1), g, gi, "geodesic",
                    ((1.3, 0.0, 0.0, 0.0), (2.7, 0.5, -0.3, 0.2)))


def lemaitre() -> Solution:
    """Schwarzschild in Lemaitre coordinates (rho, theta, phi), geodesic slicing:
    ds^2 = -dt^2 + (r_s/r) drho^2 + r^2 dOmega^2, r = (3/2 (rho - t))^(2/3) r_s^(1/3)."""
    rs = sp.Integer(1)
    rho, th = x1, x2
    r = (sp.Rational(3, 2) * (rho - t)) ** sp.Rational(2, 3) * rs ** sp.Rational(1, 3)
    g = sp.diag(rs / r, r ** 2, r ** 2 * sp.sin(th) ** 2)
    gi = sp.diag(r / rs, r ** -2, 1 / (r ** 2 * sp.sin(th) ** 2))
    return Solution("lemaitre", sp.Integer(1), g, gi, "geodesic",
                    ((0.2, 2.5, 1.0, 0.3), (0.5, 4.0, 0.7, -1.2)))


def kruskal() -> Solution:
    """Schwarzschild in Kruskal-Szekeres coordinates (X, theta, phi), zero shift:
    ds^2 = (32 M^3 / r) e^(-r/2M) (-dT^2 + dX^2) + r^2 dOmega^2 with
    r = 2M (1 + W((X^2 - T^2)/e)).  Non-constant lapse, K, D and V all non-zero.
    The lapse is given (not one of the two slicings), so the lapse equation is
    not checked for it."""
    Mm = sp.Rational(1, 2)
    Xc, th = x1, x2
    r = 2 * Mm * (1 + sp.LambertW((Xc ** 2 - t ** 2) / sp.E))
    f2 = 32 * Mm ** 3 / r * sp.exp(-r / (2 * Mm))
    g = sp.diag(f2, r ** 2, r ** 2 * sp.sin(th) ** 2)
    gi = sp.diag(1 / f2, r ** -2, 1 / (r ** 2 * sp.sin(th) ** 2))
    return Solution("kruskal", sp.sqrt(f2), g, gi, None,
                    ((0.3, 1.2, 1.0, 0.4), (-0.4, 0.9, 2.1, 0.0)))


def _shear_solution(base: Solution, name: str, points) -> Solution:
    """The same spacetime in spatial coordinates x = M x' (constant M), so that
    diagonal metrics and curvatures become fully populated."""
    sub = dict(zip(X, list(_SHEAR * sp.Matrix(X))))
    a = base.alpha.subs(sub, simultaneous=True)
    g0 = base.gamma.subs(sub, simultaneous=True)
    gi0 = base.gamma_inv.subs(sub, simultaneous=True)
    g, gi = _sheared(g0, gi0, _SHEAR)
    return Solution(name, a, g, gi, base.slicing, points)


def lemaitre_sheared() -> Solution:
    """Lemaitre coordinates followed by a constant linear change of coordinates:
    K, D and V all fully populated (tests index placement of mixed tensors)."""
    return _shear_solution(lemaitre(), "lemaitre_sheared", ((0.2, 2.1, 0.6, 0.5), (0.4, 3.3, 0.2, -0.9)))


def kruskal_sheared() -> Solution:
    """Kruskal-Szekeres followed by a constant linear change of coordinates."""
    return _shear_solution(kruskal(), "kruskal_sheared", ((0.1, 1.1, 1.3, 0.3), (-0.2, 1.2, 0.9, 0.8)))


SOLUTIONS = {
    "gauge_wave_general": gauge_wave_general,
    "two_gauge_waves": two_gauge_waves,
    "schwarzschild_isotropic_sheared": schwarzschild_isotropic_sheared,
    "kasner_sheared": kasner_sheared,
    "lemaitre": lemaitre,
    "kruskal": kruskal,
    "lemaitre_sheared": lemaitre_sheared,
    "kruskal_sheared": kruskal_sheared,
}


# --------------------------------------------------------------------------
# spacetimes with matter: every metric solves the Einstein equations with the
# energy-momentum tensor equal to its Einstein tensor (units c = 8 pi G = 1)
# --------------------------------------------------------------------------

def flrw(w) -> Solution:
    """Flat FLRW with a perfect fluid P = w rho, comoving coordinates,
    alpha = 1: a(t) = t^(2 / (3 (1 + w))), gamma = a^2 delta (section
    "Expansion of flat universe" has w = 1, gamma = t^(2/3) delta)."""
    q = sp.Rational(2, 3) / (1 + w)
    a2 = t ** (2 * q)
    name = {sp.Integer(1): "flrw_stiff", sp.Integer(0): "flrw_dust"}.get(sp.nsimplify(w), f"flrw_{w}")
    return Solution(name, sp.Integer(1), a2 * sp.eye(3), sp.eye(3) / a2, "geodesic",
                    ((1.0, 0.0, 0.0, 0.0), (1.7, 0.3, -0.2, 0.5)))


def flrw_stiff_sheared() -> Solution:
    return _shear_solution(flrw(sp.Integer(1)), "flrw_stiff_sheared", ((1.2, 0.1, 0.2, 0.3),))


def flrw_dust_sheared() -> Solution:
    return _shear_solution(flrw(sp.Integer(0)), "flrw_dust_sheared", ((1.4, -0.5, 0.2, 0.1),))


def _manufactured_metric():
    h = sp.Matrix([
        [sp.sin(x1 + t) / 8, sp.cos(x2 - 2 * t) / 15, sp.sin(x3 + x1) / 17],
        [0, sp.cos(x1 + x3 + t / 2) / 9, sp.sin(x2 - t) / 13],
        [0, 0, sp.sin(x1 - x2 + x3 + t) / 11],
    ])
    return sp.eye(3) + sp.Matrix(3, 3, lambda i, j: h[min(i, j), max(i, j)])


def manufactured() -> Solution:
    """A generic zero-shift metric (lapse and all six metric components vary
    in space and time).  Its Einstein tensor is a general energy-momentum
    tensor: energy density, momentum density G^0_k and anisotropic stresses
    are all non-zero."""
    a = 1 + sp.Rational(1, 10) * sp.sin(x1 + 2 * x2 - t / 3) + sp.Rational(1, 20) * sp.cos(x3 - t)
    g = _manufactured_metric()
    return Solution("manufactured", a, g, g.inv(method="ADJ"), None,
                    ((0.3, 0.2, -0.4, 0.7), (1.1, -0.9, 0.5, 0.2)))


def manufactured_slicing(kind: str) -> Solution:
    """The manufactured metric with a lapse that satisfies a slicing
    condition.  With zero shift tr K = -d_t ln sqrt(det gamma) / alpha, so
    d_t alpha = -alpha^2 Q holds for
      harmonic (Q = tr K):          alpha = sqrt(det gamma),
      "1+log"  (Q = tr K / alpha):  alpha = 1 + ln sqrt(det gamma)."""
    g = _manufactured_metric()
    root = sp.sqrt(g.det(method="berkowitz"))
    a = root if kind == "harmonic" else 1 + sp.log(root)
    return Solution(f"manufactured_{kind}", a, g, g.inv(method="ADJ"), kind,
                    ((0.3, 0.2, -0.4, 0.7),))


MATTER_SOLUTIONS = {
    "flrw_stiff": lambda: flrw(sp.Integer(1)),
    "flrw_dust": lambda: flrw(sp.Integer(0)),
    "flrw_stiff_sheared": flrw_stiff_sheared,
    "flrw_dust_sheared": flrw_dust_sheared,
    "manufactured": manufactured,
    "manufactured_harmonic": lambda: manufactured_slicing("harmonic"),
    "manufactured_1+log": lambda: manufactured_slicing("1+log"),
}
SOLUTIONS.update(MATTER_SOLUTIONS)


@functools.lru_cache(maxsize=None)
def _metric_derivatives(name: str):
    """Lambdified 4-metric g_ab, its first and second coordinate derivatives
    (coordinates t, x1, x2, x3; zero shift)."""
    sol = SOLUTIONS[name]()
    C = (t, x1, x2, x3)
    g4 = sp.zeros(4, 4)
    g4[0, 0] = -sol.alpha ** 2
    for i in range(3):
        for j in range(3):
            g4[1 + i, 1 + j] = sol.gamma[i, j]
    comps = [(a, b) for a in range(4) for b in range(a, 4)]
    d1 = [[sp.diff(g4[a, b], C[c]) for (a, b) in comps] for c in range(4)]
    d2 = [[[sp.diff(g4[a, b], C[c], C[d]) for (a, b) in comps] for d in range(4)] for c in range(4)]
    f0 = sp.lambdify(C, [g4[a, b] for (a, b) in comps], modules="mpmath", cse=True)
    f1 = sp.lambdify(C, d1, modules="mpmath", cse=True)
    f2 = sp.lambdify(C, d2, modules="mpmath", cse=True)
    return comps, f0, f1, f2


def einstein_matter(name: str, point):
    """The energy-momentum tensor G = Einstein tensor of the solution's
    4-metric at point, as the 10 components the sources take: G^00, G^0_k,
    G_ij (xx, xy, xz, yy, yz, zz).  Christoffel symbols and the Ricci tensor
    are formed from exact metric derivatives in 40-digit arithmetic."""
    import mpmath

    comps, f0, f1, f2 = _metric_derivatives(name)
    with mpmath.workdps(40):
        def full(vals):
            m = [[mpmath.mpf(0)] * 4 for _ in range(4)]
            for (a, b), v in zip(comps, vals):
                m[a][b] = m[b][a] = mpmath.re(v)
            return m

        g = full(f0(*point))
        dg = [full(v) for v in f1(*point)]                      # dg[c][a][b]
        ddg = [[full(v) for v in row] for row in f2(*point)]     # ddg[c][d][a][b]
        gi_m = mpmath.matrix(g) ** -1
        gi = [[gi_m[a, b] for b in range(4)] for a in range(4)]
        R4 = range(4)
        # d_e g^{ad} = -g^{ap} d_e g_pq g^{qd}
        dgi = [[[-sum(gi[a][p] * dg[e][p][q] * gi[q][d] for p in R4 for q in R4) for d in R4] for a in R4]
               for e in R4]
        # lowered Christoffel [d, bc] and its derivative
        low = [[[(dg[b][d][c] + dg[c][d][b] - dg[d][b][c]) / 2 for c in R4] for b in R4] for d in R4]
        dlow = [[[[(ddg[e][b][d][c] + ddg[e][c][d][b] - ddg[e][d][b][c]) / 2 for c in R4] for b in R4]
                 for d in R4] for e in R4]
        Gam = [[[sum(gi[a][d] * low[d][b][c] for d in R4) for c in R4] for b in R4] for a in R4]
        dGam = [[[[sum(dgi[e][a][d] * low[d][b][c] + gi[a][d] * dlow[e][d][b][c] for d in R4) for c in R4]
                  for b in R4] for a in R4] for e in R4]                 # dGam[e][a][b][c] = d_e Gam^a_bc
        Ric = [[sum(dGam[a][a][b][d] - dGam[d][a][a][b]
                    + sum(Gam[a][a][e] * Gam[e][b][d] - Gam[a][d][e] * Gam[e][a][b] for e in R4)
                    for a in R4) for d in R4] for b in R4]
        Rs = sum(gi[b][d] * Ric[b][d] for b in R4 for d in R4)
        Ein = [[Ric[a][b] - g[a][b] * Rs / 2 for b in R4] for a in R4]
        G00 = sum(gi[0][a] * gi[0][b] * Ein[a][b] for a in R4 for b in R4)
        G0k = [sum(gi[0][a] * Ein[a][1 + k] for a in R4) for k in range(3)]
        Gij = [Ein[1 + i][1 + j] for i, j in PAIRS]
        return np.array([float(v) for v in [G00] + G0k + Gij])
