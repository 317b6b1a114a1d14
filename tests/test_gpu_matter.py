"""GPU: the stress-energy hooks against the oracle.

The matter part of the sources is evaluated in the same order on both sides,
so the FP64 form agrees bit for bit: the paper's FLRW universe (a perfect
fluid given at every site and updated before every step), and seeded
per-site tensors and fluids on random states, on both lattices.
"""

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch


def _say(msg):
    print(msg, flush=True)


def _assert_equal(a, b, what):
    if not np.array_equal(a, b, equal_nan=True):
        bad = np.argwhere(~((a == b) | (np.isnan(a) & np.isnan(b))))
        raise AssertionError(f"{what}: {len(bad)} elements differ, first at {tuple(bad[0])}, "
                             f"max |diff| {np.nanmax(np.abs(a - b)):.3e}")


def test_flrw_paper_setup_bitwise():
    """Section "Expansion of flat universe": 4^3, dt = 0.001, tau = 3,
    P = rho = 1/(3 t^2), 1000 steps (t = 1 -> 2), the fluid set before every
    step and every read-out."""
    _torch()
    from paper_1505_02037_amd import lb

    dt, n_end = 1e-3, 1000
    _say("[matter] FLRW 4^3 tau=3 1000 steps")
    u0 = workloads.flrw_fields(4, 4, 4, dt)
    o = oracle.Oracle(4, 4, 4, 3.0, oracle.GEODESIC)
    with lb.Lattice(4, 4, 4, 3.0, slicing=lb.GEODESIC, device=0) as g:
        for h in (o, g):
            h.set_matter(workloads.flrw_fluid(1.0, dt), oracle.MATTER_FLUID)
            h.init_fields(u0)
        for n in range(n_end + 1):
            fl = workloads.flrw_fluid(1.0 + n * dt, dt)
            o.set_matter(fl, oracle.MATTER_FLUID)
            g.set_matter(fl, lb.MATTER_FLUID)
            if n % 100 == 0:
                _assert_equal(g.moments(), o.moments(), f"moments at step {n}")
                _assert_equal(g.distributions(), o.distributions(), f"distributions at step {n}")
            if n < n_end:
                o.step(1)
                g.step(1)
        gxx, kxx, _, _ = workloads.flrw_exact(2.0)
        u = g.moments()
        assert abs(u[1, 0, 0, 0] / gxx - 1) < 6e-5 and abs(u[7, 0, 0, 0] / (kxx * dt) - 1) < 3e-5


@pytest.mark.parametrize("lattice,shape,kind,seed,collision", [
    (19, (6, 9, 13), oracle.MATTER_TENSOR, 51, 0),
    (19, (5, 7, 11), oracle.MATTER_FLUID, 52, 0),
    (9, (1, 11, 17), oracle.MATTER_TENSOR, 53, 0),
    (9, (1, 6, 5), oracle.MATTER_FLUID, 54, 0),
    (19, (4, 6, 9), oracle.MATTER_TENSOR, 55, 1),
])
def test_per_site_matter_bitwise(lattice, shape, kind, seed, collision):
    """Seeded per-site matter on a random state, harmonic slicing, 10 steps
    (BGK, and once with the regularized collision)."""
    torch = _torch()
    from paper_1505_02037_amd import lb

    nz, ny, nx = shape
    _say(f"[matter] per-site kind={kind} lattice={lattice} {nx}x{ny}x{nz}")
    u0 = workloads.random_state(nx, ny, nz, seed=seed, amp=0.03)
    M = workloads.random_matter(nx, ny, nz, seed=seed + 100, amp=2e-3, ncomp=2 if kind else 10)
    o = oracle.Oracle(nx, ny, nz, 0.8, oracle.HARMONIC, lattice=lattice, collision=collision)
    o.set_matter(M, kind)
    o.init_fields(u0)
    with lb.Lattice(nx, ny, nz, 0.8, device=0, lattice=lattice, collision=collision) as g:
        g.set_matter(torch.from_numpy(M).cuda(), kind)  # device pointer
        g.init_fields(u0)
        for n in (0, 1, 4, 10):
            g.step(n - g.steps_done)
            o.step(n - o.steps_done)
            _assert_equal(g.distributions(), o.distributions(), f"distributions at step {n}")
            _assert_equal(g.moments(), o.moments(), f"moments at step {n}")
        # back to vacuum: the next steps equal the oracle's vacuum steps
        g.set_matter(None)
        o.set_matter(None)
        g.step(3)
        o.step(3)
        _assert_equal(g.moments(), o.moments(), "moments after returning to vacuum")


def test_uniform_tensor_and_fp32_flrw():
    """A uniform tensor (host values) bitwise, and the FP32-deviation form on
    the FLRW run within 1e-5 of the oracle (group-scaled max norm)."""
    _torch()
    from paper_1505_02037_amd import lb

    u0 = workloads.random_state(9, 5, 4, seed=61, amp=0.03)
    G = np.linspace(-1e-3, 1e-3, 10)
    o = oracle.Oracle(9, 5, 4, 0.9, oracle.GEODESIC)
    o.set_matter(G)
    o.init_fields(u0)
    o.step(6)
    with lb.Lattice(9, 5, 4, 0.9, slicing=lb.GEODESIC, device=0) as g:
        g.set_matter(G)
        g.init_fields(u0)
        g.step(6)
        _assert_equal(g.moments(), o.moments(), "uniform tensor moments")

    dt = 1e-3
    u0 = workloads.flrw_fields(4, 4, 4, dt)
    o = oracle.Oracle(4, 4, 4, 3.0, oracle.GEODESIC)
    with lb.Lattice(4, 4, 4, 3.0, slicing=lb.GEODESIC, precision=lb.FP32_DEV, device=0) as g:
        for h, kind in ((o, oracle.MATTER_FLUID), (g, lb.MATTER_FLUID)):
            h.set_matter(workloads.flrw_fluid(1.0, dt), kind)
            h.init_fields(u0)
        for n in range(1, 301):
            o.step(1)
            g.step(1)
            fl = workloads.flrw_fluid(1.0 + n * dt, dt)
            o.set_matter(fl, oracle.MATTER_FLUID)
            g.set_matter(fl, lb.MATTER_FLUID)
        ug, uo = g.moments(), o.moments()
    err_g = np.abs(ug[1:7] - uo[1:7]).max() / np.abs(uo[1:7]).max()
    err_k = np.abs(ug[7:13] - uo[7:13]).max() / np.abs(uo[7:13]).max()
    assert err_g <= 1e-5 and err_k <= 1e-5, (err_g, err_k)


def test_matter_rejected_on_fused_path():
    _torch()
    from paper_1505_02037_amd import lb

    with lb.Lattice(16, 16, 16, 0.8, device=0, path=lb.PATH_FUSED) as g:
        with pytest.raises(lb.LBError):
            g.set_matter(np.zeros(10))
        g.set_matter(None)  # vacuum is always accepted


def test_uniform_matter_changes_between_step_calls():
    """Uniform matter travels in the launch arguments: a value changed
    between step calls must reach the following steps, whichever buffer holds
    the state (odd step counts in between)."""
    _torch()
    from paper_1505_02037_amd import lb

    u0 = workloads.random_state(6, 5, 4, seed=81, amp=0.02)
    o = oracle.Oracle(6, 5, 4, 0.9, oracle.GEODESIC)
    with lb.Lattice(6, 5, 4, 0.9, slicing=lb.GEODESIC, device=0) as g:
        for h in (o, g):
            h.init_fields(u0)
        for k, n in enumerate((64, 7, 32, 33, 96)):
            G = np.full(10, 1e-4 * (k + 1))
            o.set_matter(G)
            g.set_matter(G)
            o.step(n)
            g.step(n)
            _assert_equal(g.distributions(), o.distributions(), f"distributions after call {k}")
        o.set_matter(None)
        g.set_matter(None)
        o.step(64)
        g.step(64)
        _assert_equal(g.moments(), o.moments(), "moments after returning to vacuum")
