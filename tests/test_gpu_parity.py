"""GPU parity: the HIP path against the oracle, element by element.

Both sides implement the same arithmetic in the same order without fused
multiply-add, so the FP64 form must agree bit for bit (IEEE value equality;
-0 == +0) on every distribution and every moment, at every horizon.  This is
stricter than the 1e-12 relative bound of the FP64 target, and it is what
keeps parity over long horizons: the scheme amplifies rounding differences at
the configurations' relaxation times (the grid-scale growth reaches ~1.26 per
step at tau = 0.6), so any difference in operation order would grow past
1e-12 within a few dozen steps.

Cases span several 256-thread blocks with a ragged tail, degenerate extents
(1 and 2 sites along an axis), both slicings, both lattices (D3Q19, and D2Q9
on lattices one site thick), the linear wave, and the full-size 256^3
diagonal wave (compared plane by plane with the oracle's 256 x 256 x 1 run,
which the plane symmetry of that wave makes exact).
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


def _gpu_lattice(shape, tau, slicing, path=0, lattice=19, collision=0):
    from paper_1505_02037_amd import lb

    nz, ny, nx = shape
    return lb.Lattice(nx, ny, nz, tau, slicing=slicing, device=0, path=path, lattice=lattice, collision=collision)


def _say(msg):
    print(msg, flush=True)


def _both(u0, tau, slicing, horizons, path=0, lattice=19, collision=0):
    """Yield (n, gpu moments, gpu distributions, oracle moments, oracle distributions)."""
    shape = u0.shape[1:]
    nz, ny, nx = shape
    o = oracle.Oracle(nx, ny, nz, tau, slicing, lattice=lattice, collision=collision)
    o.init_fields(u0)
    with _gpu_lattice(shape, tau, slicing, path, lattice, collision) as g:
        g.init_fields(u0)
        done = 0
        for n in horizons:
            _say(f"  step to {n} on {nx}x{ny}x{nz} tau={tau} slicing={slicing} path={path}")
            g.step(n - done)
            o.step(n - done)
            done = n
            yield n, g.moments(), g.distributions(), o.moments(), o.distributions()


def _assert_equal(a, b, what):
    if not np.array_equal(a, b, equal_nan=True):
        diff = np.abs(a - b)
        bad = np.argwhere(~((a == b) | (np.isnan(a) & np.isnan(b))))
        raise AssertionError(f"{what}: {len(bad)} elements differ, first at {tuple(bad[0])}, "
                             f"max |diff| {np.nanmax(diff):.3e}")


CASES = [
    # (name, shape (nz, ny, nx), tau, slicing, seed)
    ("random_13x7x5", (5, 7, 13), 0.7, oracle.HARMONIC, 1),
    ("random_33x17x9", (9, 17, 33), 0.6, oracle.HARMONIC, 2),
    ("random_geodesic_19x11x6", (6, 11, 19), 1.0, oracle.GEODESIC, 3),
    ("random_2x3x1", (1, 3, 2), 0.55, oracle.HARMONIC, 4),
    ("random_1x1x1", (1, 1, 1), 0.9, oracle.HARMONIC, 5),
    ("random_1x9x2", (2, 9, 1), 0.8, oracle.GEODESIC, 6),
    # several 14 x 14 tiles with ragged edges, two z-chunks (64 + 6 planes)
    ("random_33x29x70", (70, 29, 33), 0.7, oracle.HARMONIC, 7),
    ("random_geodesic_28x15x3", (3, 15, 28), 0.9, oracle.GEODESIC, 8),
    # the "1+log" slicing variant (Q = tr K / alpha)
    ("random_1pluslog_21x10x7", (7, 10, 21), 0.8, oracle.ONE_PLUS_LOG, 9),
]
PATHS = {"split": 1, "fused": 2}


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("name,shape,tau,slicing,seed", CASES, ids=[c[0] for c in CASES])
def test_random_state_bitwise(name, shape, tau, slicing, seed, path):
    _torch()
    _say(f"[parity] {name} path={path}")
    nz, ny, nx = shape
    u0 = workloads.random_state(nx, ny, nz, seed=seed, amp=0.05)
    for n, ug, fg, uo, fo in _both(u0, tau, slicing, (0, 1, 2, 10, 30), PATHS[path]):
        _assert_equal(fg, fo, f"{name} distributions at step {n}")
        _assert_equal(ug, uo, f"{name} moments at step {n}")


@pytest.mark.parametrize("path", list(PATHS))
def test_gauge_wave_1d_full_horizon(path):
    """1D gauge wave, A = 0.01, d = N = 100, tau = 0.6, ten crossings (1000
    steps): equal to the oracle at every crossing, including after the
    grid-scale instability has grown (non-finite values compared as equal)."""
    _torch()
    _say(f"[parity] gauge_wave_1d 100x1x1 tau=0.6 1000 steps path={path}")
    u0 = workloads.gauge_wave_x(100, 1, 1, 0.01, 100.0)
    for n, ug, fg, uo, fo in _both(u0, 0.6, oracle.HARMONIC, range(0, 1001, 100), PATHS[path]):
        _assert_equal(fg, fo, f"distributions at step {n}")
        _assert_equal(ug, uo, f"moments at step {n}")


@pytest.mark.parametrize("path", list(PATHS))
def test_linear_wave_bitwise(path):
    """Linear wave (geodesic slicing, A = 1e-5, tau = 4.5): exercises the
    gamma_yy/gamma_zz, K_yy/K_zz, D_xyy/D_xzz and V_x terms the gauge waves
    leave at zero."""
    _torch()
    _say(f"[parity] linear wave 40x16x15 path={path}")
    u0 = workloads.linear_wave_x(40, 16, 15, 1e-5, 40.0)
    for n, ug, fg, uo, fo in _both(u0, 4.5, oracle.GEODESIC, (1, 25, 100), PATHS[path]):
        _assert_equal(fg, fo, f"distributions at step {n}")
        _assert_equal(ug, uo, f"moments at step {n}")


CASES_D2Q9 = [
    # (name, shape (1, ny, nx), tau, slicing, seed): several blocks and a
    # ragged tail, degenerate widths, both slicings
    ("d2q9_random_37x29", (1, 29, 37), 0.7, oracle.HARMONIC, 41),
    ("d2q9_random_geodesic_300x3", (1, 3, 300), 0.9, oracle.GEODESIC, 42),
    ("d2q9_random_1x17", (1, 17, 1), 0.8, oracle.HARMONIC, 43),
    ("d2q9_random_2x1", (1, 1, 2), 0.6, oracle.HARMONIC, 44),
    ("d2q9_random_1pluslog_23x19", (1, 19, 23), 0.9, oracle.ONE_PLUS_LOG, 45),
]


@pytest.mark.parametrize("name,shape,tau,slicing,seed", CASES_D2Q9, ids=[c[0] for c in CASES_D2Q9])
def test_d2q9_random_state_bitwise(name, shape, tau, slicing, seed):
    _torch()
    _say(f"[parity] {name}")
    nz, ny, nx = shape
    u0 = workloads.random_state(nx, ny, nz, seed=seed, amp=0.05)
    for n, ug, fg, uo, fo in _both(u0, tau, slicing, (0, 1, 2, 10, 30), lattice=oracle.D2Q9):
        assert fg.shape == (16, 9) + shape
        _assert_equal(fg, fo, f"{name} distributions at step {n}")
        _assert_equal(ug, uo, f"{name} moments at step {n}")


def test_d2q9_gauge_waves_bitwise():
    """The paper's gauge-wave lattice: the x-wave (100 x 1, A = 0.01, tau =
    0.6, 1000 steps, through the blow-up) and the (1,1,0) wave on 64 x 64
    (tau = 1.0, 200 steps) equal the oracle's D2Q9 runs."""
    _torch()
    _say("[parity] d2q9 x-wave 100x1 tau=0.6 1000 steps")
    u0 = workloads.gauge_wave_x(100, 1, 1, 0.01, 100.0)
    for n, ug, fg, uo, fo in _both(u0, 0.6, oracle.HARMONIC, range(0, 1001, 200), lattice=oracle.D2Q9):
        _assert_equal(fg, fo, f"x-wave distributions at step {n}")
        _assert_equal(ug, uo, f"x-wave moments at step {n}")
    _say("[parity] d2q9 diagonal wave 64x64 tau=1.0 200 steps")
    u0 = workloads.gauge_wave_diag(64, 1, 0.1)
    for n, ug, fg, uo, fo in _both(u0, 1.0, oracle.HARMONIC, (1, 50, 200), lattice=oracle.D2Q9):
        _assert_equal(fg, fo, f"diagonal distributions at step {n}")
        _assert_equal(ug, uo, f"diagonal moments at step {n}")


@pytest.mark.parametrize("name,shape,tau,slicing,lattice", [
    ("reg_random_13x7x5", (5, 7, 13), 0.7, oracle.HARMONIC, 19),
    ("reg_random_geodesic_33x17x9", (9, 17, 33), 0.55, oracle.GEODESIC, 19),
    ("reg_d2q9_random_19x11", (1, 11, 19), 0.6, oracle.HARMONIC, 9),
])
def test_regularized_collision_bitwise(name, shape, tau, slicing, lattice):
    """The declared regularized collision equals the oracle's bit for bit."""
    _torch()
    _say(f"[parity] {name}")
    nz, ny, nx = shape
    u0 = workloads.random_state(nx, ny, nz, seed=71, amp=0.05)
    for n, ug, fg, uo, fo in _both(u0, tau, slicing, (1, 2, 10, 30), lattice=lattice,
                                   collision=oracle.COLLISION_REGULARIZED):
        _assert_equal(fg, fo, f"{name} distributions at step {n}")
        _assert_equal(ug, uo, f"{name} moments at step {n}")


def test_regularized_gauge_wave_1d_long_horizon():
    """1D gauge wave, A = 0.01, tau = 0.6, 1000 steps with the regularized
    collision (which outlives BGK's blow-up): equal to the oracle throughout."""
    _torch()
    _say("[parity] regularized gauge wave 100x1x1 tau=0.6 1000 steps")
    u0 = workloads.gauge_wave_x(100, 1, 1, 0.01, 100.0)
    for n, ug, fg, uo, fo in _both(u0, 0.6, oracle.HARMONIC, range(0, 1001, 200),
                                   collision=oracle.COLLISION_REGULARIZED):
        _assert_equal(fg, fo, f"distributions at step {n}")
        _assert_equal(ug, uo, f"moments at step {n}")


def test_regularized_rejected_on_fused_path():
    _torch()
    from paper_1505_02037_amd import lb

    with pytest.raises(lb.LBError):
        lb.Lattice(16, 16, 16, 0.8, device=0, path=lb.PATH_FUSED, collision=lb.COLLISION_REGULARIZED)


def test_gauge_wave_3d_x_128_resolution_pieces():
    """x-wave on 64 x 8 x 8 (a 3D lattice) equals the oracle at several
    horizons at each tau of the 3D gauge-wave series."""
    _torch()
    for tau in (0.55, 0.6, 1.0):
        _say(f"[parity] x-wave 64x8x8 tau={tau}")
        u0 = workloads.gauge_wave_x(64, 8, 8, 0.1, 64.0)
        for n, ug, fg, uo, fo in _both(u0, tau, oracle.HARMONIC, (1, 20, 64)):
            _assert_equal(ug, uo, f"tau={tau} moments at step {n}")


def test_diagonal_wave_256_cubed_plane_by_plane():
    """Full-size 256^3 (1,1,0) wave, A = 0.1, tau = 0.6, FP64 (the benchmark's
    workload and launch configuration): after a few steps every z-plane of the
    GPU moments equals the oracle's 256 x 256 x 1 run, and the error norms
    kernel agrees with numpy."""
    torch = _torch()
    n, steps = 256, 3
    _say(f"[parity] diagonal wave {n}^3 tau=0.6 steps={steps}")
    u2 = workloads.gauge_wave_diag(n, 1, 0.1)
    o = oracle.Oracle(n, n, 1, 0.6)
    o.init_fields(u2)
    o.step(steps)
    uo = o.moments()[:, 0]
    u3 = torch.from_numpy(u2).cuda().expand(16, n, n, n).contiguous()
    with _gpu_lattice((n, n, n), 0.6, oracle.HARMONIC) as g:  # the default path, as benchmarked
        g.init_fields(u3)
        del u3
        g.step(steps)
        ug = torch.empty((16, n, n, n), dtype=torch.float64, device="cuda")
        g.moments(ug)
        for z in range(0, n, 17):
            _assert_equal(ug[:, z].cpu().numpy(), uo, f"plane z={z}")
        same = bool((ug == ug[:, :1]).all().item())
        assert same, "GPU 256^3 result is not z-invariant"
        # error norms against the analytic wave at t = steps
        ua = torch.from_numpy(workloads.gauge_wave_diag(n, 1, 0.1, t=steps)).cuda().expand(16, n, n, n).contiguous()
        norms = g.error_norms(ua)
        d = (ug - ua).abs().amax(dim=(1, 2, 3)).cpu().numpy()
        assert np.array_equal(norms["max_abs"], d)
        l2 = torch.sqrt(((ug - ua) ** 2).mean(dim=(1, 2, 3))).cpu().numpy()
        assert np.allclose(norms["l2"], l2, rtol=1e-12, atol=0)


@pytest.mark.parametrize("path,collision,slicing", [
    ("split", 0, oracle.HARMONIC), ("fused", 0, oracle.HARMONIC),
    ("split", 1, oracle.HARMONIC), ("split", 0, oracle.ONE_PLUS_LOG),
], ids=["split", "fused", "split-regularized", "split-1pluslog"])
def test_random_state_256_cubed_sampled_sites(path, collision, slicing):
    """The benchmark's lattice size and launch configuration with a random,
    not plane-symmetric, state: after two steps the moments and distributions
    at sampled sites (corners and faces, where the periodic wrap acts, and
    random sites) equal the oracle's bit for bit, the oracle evolving a
    periodic window around each site (exact by locality, pinned in
    tests/test_oracle_windows.py)."""
    torch = _torch()
    import oracle_windows as ow
    from paper_1505_02037_amd import lb

    n, steps, tau = 256, 2, 0.6
    _say(f"[parity] random state {n}^3 path={path} collision={collision} slicing={slicing}, "
         f"sampled sites after {steps} steps")
    u0 = workloads.random_state(n, n, n, seed=256, amp=0.05)
    cs = ow.sample_centres(n, 18, seed=257)
    uo, fo = ow.sampled(u0, cs, tau, steps, slicing=slicing, collision=collision)
    iz, iy, ix = (torch.tensor([c[k] for c in cs], device="cuda") for k in range(3))
    with lb.Lattice(n, n, n, tau, slicing=slicing, device=0, path=PATHS[path], collision=collision) as g:
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
    _assert_equal(us, uo, "moments at sampled sites")
    _assert_equal(fs, fo, "distributions at sampled sites")


def test_largest_fp64_lattice_random_state_sampled_sites():
    """The largest cubic FP64 lattice the card holds (edge ~376), random
    state: after two steps the moments at sampled sites (corners, faces,
    random sites) equal the windowed oracle's bit for bit."""
    torch = _torch()
    import oracle_windows as ow
    from gpu_sizing import largest_edge
    from paper_1505_02037_amd import lb

    e = largest_edge(torch, lb.FP64, lo=128, hi=512)
    steps, tau = 2, 0.6
    _say(f"[parity] largest FP64 lattice {e}^3 ({e ** 3 / 1e6:.0f} M sites), random state, sampled sites")
    u0 = workloads.random_state(e, e, e, seed=376, amp=0.05)
    cs = ow.sample_centres(e, 18, seed=377)
    uo, _ = ow.sampled(u0, cs, tau, steps)
    iz, iy, ix = (torch.tensor([c[k] for c in cs], device="cuda") for k in range(3))
    with lb.Lattice(e, e, e, tau, device=0) as g:
        g.init_fields(u0)
        del u0
        g.step(steps)
        u = torch.empty((16, e, e, e), dtype=torch.float64, device="cuda")
        g.moments(u)
        us = u[:, iz, iy, ix].cpu().numpy()
        del u
    torch.cuda.empty_cache()
    _assert_equal(us, uo, f"moments at sampled sites of {e}^3")


def test_error_norms_small():
    torch = _torch()
    _say("[parity] error norms 9x8x7")
    u0 = workloads.random_state(9, 8, 7, seed=9)
    ref = workloads.random_state(9, 8, 7, seed=10)
    with _gpu_lattice((7, 8, 9), 0.8, oracle.HARMONIC) as g:
        g.init_fields(u0)
        g.step(2)
        u = g.moments()
        nr = g.error_norms(ref)
        nd = g.error_norms(torch.from_numpy(ref).cuda())
    d = np.abs(u - ref).reshape(16, -1)
    assert np.array_equal(nr["max_abs"], d.max(axis=1))
    assert np.allclose(nr["l2"], np.sqrt((d ** 2).mean(axis=1)), rtol=1e-13, atol=0)
    assert np.array_equal(nr["ref_max"], np.abs(ref).reshape(16, -1).max(axis=1))
    for k in nr:
        assert np.array_equal(nr[k], nd[k])


def test_device_pointers_and_stream():
    """Inputs and outputs as device tensors on a caller-owned stream."""
    torch = _torch()
    _say("[parity] device pointers on a torch stream")
    from paper_1505_02037_amd import lb

    u0 = workloads.random_state(10, 6, 4, seed=12)
    s = torch.cuda.Stream()
    with lb.Lattice(10, 6, 4, 0.75, device=0, stream=s.cuda_stream) as g:
        with torch.cuda.stream(s):
            du = torch.from_numpy(u0).cuda()
        s.synchronize()
        g.init_fields(du)
        g.step(5)
        out = torch.empty_like(du)
        g.moments(out)
        fo = torch.empty((16, 19, 4, 6, 10), dtype=torch.float64, device="cuda")
        g.distributions(fo)
        assert g.steps_done == 5
    o = oracle.Oracle(10, 6, 4, 0.75)
    o.init_fields(u0)
    o.step(5)
    _assert_equal(out.cpu().numpy(), o.moments(), "moments")
    _assert_equal(fo.cpu().numpy(), o.distributions(), "distributions")


def test_kernel_timing_names_the_launched_kernels():
    _torch()
    from paper_1505_02037_amd import lb

    cases = (
        (19, 32, 1, {"lbnr::k_moments<lbnr::D3Q19>", "lbnr::k_collide<lbnr::D3Q19, false, 0>"}),
        (19, 32, 2, {"lbnr::k_fused<double>"}),
        (9, 1, 1, {"lbnr::k_moments<lbnr::D2Q9>", "lbnr::k_collide<lbnr::D2Q9, false, 0>"}),
    )
    for lattice, nz, path, names in cases:
        with lb.Lattice(32, 32, nz, 0.6, device=0, path=path, lattice=lattice) as g:
            g.init_fields(workloads.gauge_wave_x(32, 32, nz, 0.1, 32))
            g.set_timing(True)
            g.step(3)
            t = g.kernel_times()
        assert set(t) == names
        assert all(v > 0 for v in t.values())


def test_timed_steps_span_chunks_and_change_nothing():
    """A timed call longer than one timing chunk (256 steps) gives the untimed
    call's state bit for bit, and per-launch times averaged over all steps."""
    _torch()
    from paper_1505_02037_amd import lb

    u0 = workloads.gauge_wave_x(12, 6, 5, 0.05, 12)
    res = []
    for path, timed in ((1, False), (1, True), (2, True)):
        with lb.Lattice(12, 6, 5, 1.0, device=0, path=path) as g:
            g.init_fields(u0)
            g.set_timing(timed)
            g.step(600)
            if timed:
                t = g.kernel_times()
                assert len(t) == (2 if path == 1 else 1) and all(v > 0 for v in t.values())
            res.append(g.distributions())
    assert np.array_equal(res[0], res[1], equal_nan=True)
    assert np.array_equal(res[0], res[2], equal_nan=True)


def test_fused_and_split_paths_agree_after_moments_calls():
    """Interleaving output calls (which recompute the moments) with fused steps
    leaves the evolution unchanged."""
    _torch()
    from paper_1505_02037_amd import lb

    u0 = workloads.random_state(30, 16, 9, seed=31)
    res = []
    for path, probe in ((1, False), (2, False), (2, True)):
        with lb.Lattice(30, 16, 9, 0.7, device=0, path=path) as g:
            g.init_fields(u0)
            for _ in range(4):
                g.step(3)
                if probe:
                    g.moments()
            res.append(g.distributions())
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[1], res[2])
