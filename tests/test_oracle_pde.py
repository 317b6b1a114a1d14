"""Pin the oracle's Bona-Masso right-hand sides with exact vacuum solutions.

For each exact solution the point routine of the oracle is evaluated on the
analytic state (alpha, gamma, K, V, A, D), and the evolution equations of the
section "Bona-Masso evolution equations" must hold:

    d_t alpha = R_alpha (slicing of the solution), d_t gamma = R_gamma,
    d_t K_ij + d_k(alpha lambda^k_ij) = alpha S_ij,  d_t V_k = Omega_k.

The time derivatives are exact (sympy); the flux divergence is a 6th-order
central difference of the oracle's own flux evaluated on the analytic state.
The solution set activates every term of S_ij, Omega_k and lambda^k_ij with a
fully populated metric (sheared coordinates), including cross terms between
A, D, K and V (Kruskal-Szekeres, Lemaitre).  A planted sign flip, dropped term
or transposed index in any of those formulas breaks at least one case.

Reading used (the printed equation does not hold otherwise): in the bracket
multiplying gamma_ij/4 of S_ij, the factor D_s^{ks} is read as D^{ks}_s, the
trace D_sr^r with its free index raised.
"""

import numpy as np
import pytest

import oracle

es = pytest.importorskip("exact_solutions")

H = 1e-3
FD6 = {-3: -1.0, -2: 9.0, -1: -45.0, 1: 45.0, 2: -9.0, 3: 1.0}


def _rhs(st, slicing):
    return oracle.point_rhs(st[0], st[1:7], st[7:13], st[13:16], st[16:19], st[19:37], slicing)


def _flux_divergence(name, P, slicing):
    div = np.zeros(6)
    for k in range(3):
        acc = np.zeros(6)
        for m, cm in FD6.items():
            Q = list(P)
            Q[1 + k] += m * H
            st, _ = es.evaluate(name, Q)
            acc += cm * st[0] * _rhs(st, slicing)["lambda"][k]
        div += acc / (60.0 * H)
    return div


CASES = [
    ("gauge_wave_general", 0), ("gauge_wave_general", 1), ("gauge_wave_general", 2),
    ("two_gauge_waves", 0), ("two_gauge_waves", 1),
    ("schwarzschild_isotropic_sheared", 0), ("schwarzschild_isotropic_sheared", 1),
    ("kasner_sheared", 0), ("kasner_sheared", 1),
    ("lemaitre", 0), ("lemaitre", 1),
    ("kruskal", 0), ("kruskal", 1),
    ("lemaitre_sheared", 0),
    ("kruskal_sheared", 0),
]


@pytest.mark.parametrize("name,ip", CASES)
def test_exact_solution_satisfies_oracle_equations(name, ip):
    sol, _, _ = es.compiled(name)
    P = sol.points[ip]
    slicing = oracle.HARMONIC if sol.slicing == "harmonic" else oracle.GEODESIC
    st, dt = es.evaluate(name, P)
    r = _rhs(st, slicing)
    scale = 1.0 + max(np.abs(dt).max(), np.abs(r["R_K"]).max(), np.abs(r["Omega"]).max())
    tol = 1e-10 * scale

    # three-metric equation (zero shift)
    assert np.abs(dt[1:7] - r["R_gamma"]).max() <= tol
    # slicing condition, when the solution is in one of the two slicings
    if sol.slicing is not None:
        assert abs(dt[0] - r["R_alpha"]) <= tol
    # momentum-variable equation (its flux vanishes at zero shift)
    assert np.abs(dt[13:16] - r["Omega"]).max() <= tol
    # extrinsic-curvature equation in flux-conservative form
    div = _flux_divergence(name, P, slicing)
    res = dt[7:13] + div - r["R_K"]
    assert np.abs(res).max() <= 1e-9 * scale, res


def test_solutions_are_not_trivial():
    """The K, D, V, A content of the set (guards the pins against vacuity)."""
    seen = {"K": 0.0, "D": 0.0, "V": 0.0, "A": 0.0, "KD": 0.0, "AK": 0.0, "offdiag": 0.0}
    for name, ip in CASES:
        sol, _, _ = es.compiled(name)
        st, _ = es.evaluate(name, sol.points[ip])
        K, V, A, D = st[7:13], st[13:16], st[16:19], st[19:37]
        seen["K"] = max(seen["K"], np.abs(K).max())
        seen["V"] = max(seen["V"], np.abs(V).max())
        seen["A"] = max(seen["A"], np.abs(A).max())
        seen["D"] = max(seen["D"], np.abs(D).max())
        seen["KD"] = max(seen["KD"], min(np.abs(K).max(), np.abs(D).max(), np.abs(V).max()))
        seen["AK"] = max(seen["AK"], min(np.abs(K).max(), np.abs(A).max(), np.abs(V).max()))
        seen["offdiag"] = max(seen["offdiag"], min(abs(K[1]), abs(st[2]), abs(D[1])))
    for k, v in seen.items():
        assert v > 1e-2, (k, v)


# --------------------------------------------------------------------------
# matter: the energy-momentum terms of S_ij and Omega_k
# --------------------------------------------------------------------------

MATTER_CASES = [
    ("flrw_stiff", 0), ("flrw_stiff", 1), ("flrw_dust", 1),
    ("flrw_stiff_sheared", 0), ("flrw_dust_sheared", 0),
    ("manufactured", 0), ("manufactured", 1),
    ("manufactured_1+log", 0),
]
SLICING = {"harmonic": oracle.HARMONIC, "geodesic": oracle.GEODESIC, "1+log": oracle.ONE_PLUS_LOG, None: oracle.GEODESIC}


def test_einstein_tensor_helper_gives_the_friedmann_fluid():
    """The helper that turns a metric into its energy-momentum tensor is
    itself pinned by the Friedmann equations: for a = t^(1/3) (the paper's
    stiff fluid) G^00 = rho = P = 1/(3 t^2) and G_ij = P gamma_ij; for dust,
    a = t^(2/3), rho = 4/(3 t^2) and P = 0; vacuum solutions give zero."""
    for tt in (1.0, 1.7):
        G = es.einstein_matter("flrw_stiff", (tt, 0.1, 0.2, 0.3))
        rho = 1.0 / (3.0 * tt * tt)
        g = tt ** (2.0 / 3.0)
        assert np.allclose(G, [rho, 0, 0, 0, rho * g, 0, 0, rho * g, 0, rho * g], rtol=1e-14, atol=1e-15)
        G = es.einstein_matter("flrw_dust", (tt, 0.1, 0.2, 0.3))
        assert np.allclose(G, [4.0 / (3.0 * tt * tt)] + [0.0] * 9, rtol=1e-14, atol=1e-15)
    for name in ("schwarzschild_isotropic_sheared", "kasner_sheared"):
        sol, _, _ = es.compiled(name)
        assert np.abs(es.einstein_matter(name, sol.points[0])).max() < 1e-14


@pytest.mark.parametrize("name,ip", MATTER_CASES)
def test_matter_solution_satisfies_oracle_equations(name, ip):
    """Every metric solves the Einstein equations with the energy-momentum
    tensor taken as its Einstein tensor; with that matter the oracle's
    sources must satisfy the evolution equations point-wise.  The FLRW cases
    carry the paper's fluid (isotropic pressure, energy density); the
    manufactured spacetime has momentum density G^0_k and anisotropic
    stresses, with a varying lapse; its "1+log" variant takes the lapse that
    slicing condition fixes, which pins the "1+log" lapse equation (section
    "Gauge choices") on a generic metric (the harmonic one is pinned by the
    gauge waves)."""
    sol, _, _ = es.compiled(name)
    P = sol.points[ip]
    st, dt = es.evaluate(name, P)
    G = es.einstein_matter(name, P)
    slicing = SLICING[sol.slicing]
    r = oracle.point_rhs(st[0], st[1:7], st[7:13], st[13:16], st[16:19], st[19:37], slicing, matter=G)
    vac = _rhs(st, slicing)
    scale = 1.0 + max(np.abs(dt).max(), np.abs(r["R_K"]).max(), np.abs(r["Omega"]).max())
    tol = 1e-10 * scale
    assert np.abs(dt[1:7] - r["R_gamma"]).max() <= tol
    if sol.slicing is not None:
        assert abs(dt[0] - r["R_alpha"]) <= tol
        if sol.slicing != "geodesic":
            assert abs(dt[0]) > 1e-3  # the lapse equation is exercised
    assert np.abs(dt[13:16] - r["Omega"]).max() <= tol
    div = _flux_divergence(name, P, slicing)
    assert np.abs(dt[7:13] + div - r["R_K"]).max() <= 1e-9 * scale
    # the matter terms are not vacuous for these cases.  For dust the energy
    # density's two terms in S_ij (from -R4_ij and from the bracket) cancel,
    # so the dust cases pin that cancellation rather than a net source.
    if not name.startswith("flrw_dust"):
        assert np.abs(dt[7:13] + div - vac["R_K"]).max() > 1e-3 or np.abs(dt[13:16] - vac["Omega"]).max() > 1e-3


def test_manufactured_matter_is_general():
    """Guard against vacuity: the manufactured spacetime's matter has energy
    density, momentum density and off-diagonal stress."""
    G = es.einstein_matter("manufactured", es.SOLUTIONS["manufactured"]().points[0])
    assert abs(G[0]) > 1e-2 and np.abs(G[1:4]).min() > 1e-3 and np.abs(G[[5, 6, 8]]).max() > 1e-2
