"""The windowed oracle (tests/oracle_windows.py) against the oracle run on the
whole lattice: the locality bound behind the sampled full-size parity tests."""

import numpy as np
import pytest

import oracle
import oracle_windows as ow
import workloads

CENTRES = [(0, 0, 0), (14, 16, 19), (7, 0, 19), (3, 9, 11)]


@pytest.mark.parametrize("steps", [1, 2, 3])
def test_window_centre_equals_whole_lattice(steps):
    nx, ny, nz = 20, 17, 15
    u0 = workloads.random_state(nx, ny, nz, seed=3, amp=0.05)
    o = oracle.Oracle(nx, ny, nz, 0.6)
    o.init_fields(u0)
    o.step(steps)
    U, F = o.moments(), o.distributions()
    us, fs = ow.sampled(u0, CENTRES, 0.6, steps)
    for i, (z, y, x) in enumerate(CENTRES):
        assert np.array_equal(us[:, i], U[:, z, y, x]), (steps, i)
        assert np.array_equal(fs[:, :, i], F[:, :, z, y, x]), (steps, i)
    # the bound is tight: one site less and the window's wrap reaches the
    # centre's moments
    us_small, _ = ow.sampled(u0, CENTRES, 0.6, steps, R=ow.window_radius(steps) - 1)
    assert not all(np.array_equal(us_small[:, i], U[:, z, y, x]) for i, (z, y, x) in enumerate(CENTRES))


@pytest.mark.parametrize("collision,slicing", [(oracle.COLLISION_REGULARIZED, oracle.HARMONIC),
                                               (oracle.COLLISION_BGK, oracle.ONE_PLUS_LOG)])
def test_window_centre_equals_whole_lattice_variants(collision, slicing):
    nx, ny, nz = 18, 16, 15
    u0 = workloads.random_state(nx, ny, nz, seed=4, amp=0.05)
    o = oracle.Oracle(nx, ny, nz, 0.6, slicing, collision=collision)
    o.init_fields(u0)
    o.step(2)
    U, F = o.moments(), o.distributions()
    us, fs = ow.sampled(u0, CENTRES[:1] + [(14, 15, 17), (7, 0, 9)], 0.6, 2, slicing=slicing, collision=collision)
    for i, (z, y, x) in enumerate(CENTRES[:1] + [(14, 15, 17), (7, 0, 9)]):
        assert np.array_equal(us[:, i], U[:, z, y, x]), i
        assert np.array_equal(fs[:, :, i], F[:, :, z, y, x]), i
