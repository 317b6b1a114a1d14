"""GPU: the FP32-deviation form against the FP64 oracle.

Distributions are stored as FP32 deviations from the rest-state equilibrium
and relaxed in FP32; the moments, geometry, sources and flux are FP64.  The
bound is the one the FP32 form is built to: the value-relative max-norm error
of every field (max |u - u_oracle| / max |u_oracle|) stays at or below 1e-5.
At tau = 0.6 the scheme's grid-scale growth (~1.26 per step) amplifies the
FP32 rounding, so the bound is checked over the horizon it can hold (a few
tens of steps); at larger tau it holds for hundreds of steps.
"""

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _torch():
    import torch

    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch


def _rel_err(u, ref):
    """Per field: max |u - ref| over the lattice divided by the max-norm of the
    field's tensor (alpha alone; all gamma components; K and V together,
    both of dimension 1/length).  Components that vanish analytically carry
    only rounding noise in the reference, so their own max would not be a
    scale."""
    m = np.abs(ref).reshape(16, -1).max(axis=1)
    scale = np.empty(16)
    scale[0] = m[0]
    scale[1:7] = m[1:7].max()
    scale[7:16] = m[7:16].max()
    num = np.abs(u - ref).reshape(16, -1).max(axis=1)
    return num / scale


def _fp32(shape, tau, slicing=oracle.HARMONIC, lattice=19, collision=0):
    from paper_1505_02037_amd import lb

    nz, ny, nx = shape
    return lb.Lattice(nx, ny, nz, tau, slicing=slicing, precision=lb.FP32_DEV, device=0, lattice=lattice,
                      collision=collision)


@pytest.mark.parametrize("shape,tau,slicing,seed,horizons,lattice,collision", [
    ((5, 7, 13), 0.7, oracle.HARMONIC, 1, (0, 1, 5, 10), 19, 0),
    ((9, 17, 33), 1.0, oracle.GEODESIC, 2, (0, 1, 10, 30), 19, 0),
    ((1, 3, 2), 0.9, oracle.HARMONIC, 3, (0, 2, 10), 19, 0),
    ((1, 29, 37), 0.8, oracle.HARMONIC, 4, (0, 1, 5, 10), 9, 0),
    ((1, 1, 5), 1.0, oracle.GEODESIC, 5, (0, 2, 10), 9, 0),
    ((5, 7, 13), 0.7, oracle.HARMONIC, 6, (0, 1, 5, 10), 19, 1),
])
def test_fp32_random_state_within_bound(shape, tau, slicing, seed, horizons, lattice, collision):
    _torch()
    nz, ny, nx = shape
    print(f"[fp32] random {nx}x{ny}x{nz} tau={tau} lattice=D{2 if lattice == 9 else 3}Q{lattice} "
          f"collision={collision}", flush=True)
    u0 = workloads.random_state(nx, ny, nz, seed=seed, amp=0.05)
    o = oracle.Oracle(nx, ny, nz, tau, slicing, lattice=lattice, collision=collision)
    o.init_fields(u0)
    with _fp32(shape, tau, slicing, lattice, collision) as g:
        g.init_fields(u0)
        done = 0
        for n in horizons:
            g.step(n - done)
            o.step(n - done)
            done = n
            err = _rel_err(g.moments(), o.moments())
            assert err.max() <= TOL, (n, err)
            fd = np.abs(g.distributions() - o.distributions()).max()
            assert fd <= TOL * 0.1, (n, fd)


def test_fp32_x_wave_long_horizon_at_tau_1():
    """x-wave, A = 0.1, d = 64, tau = 1.0.  The FP32 storage of the metric
    deviation limits the derivative stencil to ~1e-6 relative (neighbour
    differences of gamma are ~1e-2 of values stored to 6e-8), and the scheme's
    growth at tau = 1 amplifies it: 1e-5 holds to 100 steps, 1e-4 to 200."""
    _torch()
    print("[fp32] x-wave 64x4x4 tau=1.0, 200 steps", flush=True)
    u0 = workloads.gauge_wave_x(64, 4, 4, 0.1, 64)
    o = oracle.Oracle(64, 4, 4, 1.0)
    o.init_fields(u0)
    with _fp32((4, 4, 64), 1.0) as g:
        g.init_fields(u0)
        for n, bound in ((50, TOL), (100, TOL), (200, 10 * TOL)):
            g.step(50 if n <= 100 else 100)
            o.step(50 if n <= 100 else 100)
            err = _rel_err(g.moments(), o.moments())
            assert err.max() <= bound, (n, err)


def test_fp32_diagonal_256_cubed():
    """The 256^3 benchmark workload in the FP32 form: (1,1,0) wave,
    A = 0.1, tau = 0.6.  Every z-plane equals the others bit for bit, and the
    fields stay within 1e-5 of the FP64 oracle (256 x 256 x 1, exact by the
    wave's plane symmetry) for the first steps; after that the FP32 floor of
    the stored lapse/metric deviations (~3e-8 absolute on values near 1, i.e.
    ~1e-5 of the neighbour differences over a 181-site wavelength) reaches K
    through the derivative stencil and the scheme's growth, so the bound at
    10 steps is 1e-4 (alpha, gamma and V stay below 1e-7)."""
    torch = _torch()
    n = 256
    print(f"[fp32] diagonal wave {n}^3 tau=0.6", flush=True)
    u2 = workloads.gauge_wave_diag(n, 1, 0.1)
    o = oracle.Oracle(n, n, 1, 0.6)
    o.init_fields(u2)
    with _fp32((n, n, n), 0.6) as g:
        g.init_fields(torch.from_numpy(u2).cuda().expand(16, n, n, n).contiguous())
        ug = torch.empty((16, n, n, n), dtype=torch.float64, device="cuda")
        for steps, total, bound in ((1, 1, TOL), (1, 2, TOL), (8, 10, 10 * TOL)):
            g.step(steps)
            o.step(steps)
            g.moments(ug)
            assert bool((ug == ug[:, :1]).all().item())
            err = _rel_err(ug[:, 0].cpu().numpy(), o.moments()[:, 0])
            print(f"  step {total}: max value-relative error {err.max():.3e} (field {err.argmax()})", flush=True)
            assert err.max() <= bound, (total, err)
            assert max(err[0], err[1:7].max(), err[13:16].max()) <= 1e-7, (total, err)


def test_fp32_random_state_256_cubed_sampled_sites():
    """The FP32 form at the benchmark's lattice size with a random state:
    after two steps the moments at sampled sites (corners, faces, random
    sites) are within the FP32 bound of the FP64 oracle evolved on a window
    around each site, and so are the distributions (a tenth of it)."""
    torch = _torch()
    import oracle_windows as ow

    n, steps, tau = 256, 2, 0.6
    print(f"[fp32] random state {n}^3, sampled sites after {steps} steps", flush=True)
    u0 = workloads.random_state(n, n, n, seed=258, amp=0.05)
    cs = ow.sample_centres(n, 18, seed=259)
    uo, fo = ow.sampled(u0, cs, tau, steps)
    iz, iy, ix = (torch.tensor([c[k] for c in cs], device="cuda") for k in range(3))
    with _fp32((n, n, n), tau) as g:
        g.init_fields(u0)
        del u0
        g.step(steps)
        ug = torch.empty((16, n, n, n), dtype=torch.float64, device="cuda")
        g.moments(ug)
        us = ug[:, iz, iy, ix].cpu().numpy()
        del ug
        fg = torch.empty((16, 19, n, n, n), dtype=torch.float64, device="cuda")
        g.distributions(fg)
        fs = fg[:, :, iz, iy, ix].cpu().numpy()
        del fg
    torch.cuda.empty_cache()
    err = _rel_err(us, uo)
    assert err.max() <= TOL, err
    assert np.abs(fs - fo).max() <= TOL * 0.1


def test_fp32_fused_equals_split_bitwise():
    """The FP32 form's one-launch and two-launch steps run the same arithmetic."""
    _torch()
    from paper_1505_02037_amd import lb

    u0 = workloads.random_state(31, 29, 70, seed=12)
    out = []
    for path in (1, 2):
        with lb.Lattice(31, 29, 70, 0.8, precision=lb.FP32_DEV, device=0, path=path) as g:
            g.init_fields(u0)
            g.step(7)
            out.append((g.moments(), g.distributions()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_fp32_error_norms_and_kernel_names():
    torch = _torch()
    u0 = workloads.random_state(12, 10, 8, seed=4)
    ref = workloads.random_state(12, 10, 8, seed=5)
    with _fp32((8, 10, 12), 0.8) as g:
        g.init_fields(u0)
        g.set_timing(True)
        g.step(2)
        assert set(g.kernel_times()) == {"lbnr::k_moments32<lbnr::D3Q19>", "lbnr::k_collide32<lbnr::D3Q19, false, 0>"}
        u = g.moments()
        nr = g.error_norms(torch.from_numpy(ref).cuda())
    assert np.array_equal(nr["max_abs"], np.abs(u - ref).reshape(16, -1).max(axis=1))


def _largest_edge(torch):
    """Edge (256..488) of the largest cubic FP32 lattice that fits the free
    device memory beside one 16-field FP64 moments array and a margin."""
    from gpu_sizing import largest_edge
    from paper_1505_02037_amd import lb

    return largest_edge(torch, lb.FP32_DEV)


def test_largest_fp32_lattice_rows_match_oracle():
    """The largest configuration's launch shape: an FP32-deviation lattice
    sized to fill the card (edge up to 488), x-wave A = 0.05, tau = 0.6.
    After two steps every (y, z) row is identical (bitwise) and equals the
    oracle's one-dimensional FP64 run within the FP32 bound."""
    torch = _torch()
    from paper_1505_02037_amd import lb

    e = _largest_edge(torch)
    print(f"[fp32] largest lattice {e}^3 ({e ** 3 / 1e6:.0f} M sites)", flush=True)
    A, tau, steps = 0.05, 0.6, 2
    row = torch.from_numpy(workloads.gauge_wave_x(e, 1, 1, A, float(e)))
    u = row.cuda().expand(16, e, e, e).contiguous()
    with lb.Lattice(e, e, e, tau, precision=lb.FP32_DEV, device=0) as g:
        g.init_fields(u)
        g.step(steps)
        g.moments(u)  # the input tensor is reused for the output
    same = bool((u == u[:, :1, :1, :]).all().item())
    assert same, "rows of the plane-symmetric wave differ"
    o = oracle.Oracle(e, 1, 1, tau)
    o.init_fields(workloads.gauge_wave_x(e, 1, 1, A, float(e)))
    o.step(steps)
    err = _rel_err(u[:, :1, :1, :].cpu().numpy(), o.moments())
    del u
    assert err.max() <= TOL, err


def test_largest_fp32_lattice_random_state_sampled_sites():
    """The largest lattice with a random, not plane-symmetric, state (64-bit
    offsets of every field and direction in use): after two steps the moments
    at sampled sites are within the FP32 bound of the FP64 oracle evolved on a
    window around each site."""
    torch = _torch()
    import oracle_windows as ow
    from paper_1505_02037_amd import lb

    e = _largest_edge(torch)
    steps, tau = 2, 0.6
    print(f"[fp32] largest lattice {e}^3, random state, sampled sites after {steps} steps", flush=True)
    u0 = workloads.random_state(e, e, e, seed=488, amp=0.05)
    cs = ow.sample_centres(e, 18, seed=489)
    uo, _ = ow.sampled(u0, cs, tau, steps)
    iz, iy, ix = (torch.tensor([c[k] for c in cs], device="cuda") for k in range(3))
    with lb.Lattice(e, e, e, tau, precision=lb.FP32_DEV, device=0) as g:
        g.init_fields(u0)
        del u0
        g.step(steps)
        u = torch.empty((16, e, e, e), dtype=torch.float64, device="cuda")
        g.moments(u)
        us = u[:, iz, iy, ix].cpu().numpy()
        del u
    torch.cuda.empty_cache()
    err = _rel_err(us, uo)
    assert err.max() <= TOL, err
