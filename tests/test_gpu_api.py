"""GPU: error paths and state rules of the C-ABI (every call here returns an
error code from host-side checks or from a HIP call that fails cleanly)."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _lb():
    import torch

    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1505_02037_amd import lb

    return lb


def test_state_rules():
    lb = _lb()
    with lb.Lattice(8, 6, 4, 0.8, device=0) as g:
        with pytest.raises(lb.LBError, match="not initialised"):
            g.moments()
        with pytest.raises(lb.LBError, match="not initialised"):
            g.step(1)
        with pytest.raises(lb.LBError):
            g.kernel_times()          # no timed step yet
        g.init_fields(workloads.random_state(8, 6, 4, seed=1))
        with pytest.raises(lb.LBError, match="invalid"):
            g.step(-1)
        g.step(0)
        assert g.steps_done == 0
        g.step(2)
        assert g.steps_done == 2
        with pytest.raises(lb.LBError, match="invalid"):
            g.set_matter(np.zeros(10), kind=5)
        with pytest.raises(ValueError):
            g.init_fields(np.zeros((16, 4, 6, 9)))   # wrong shape: refused before the call
        u = g.moments()
        assert np.all(np.isfinite(u))
        g.init_fields(workloads.random_state(8, 6, 4, seed=1))   # re-initialisation resets the counter
        assert g.steps_done == 0


def test_bad_device_is_an_error_not_a_fault():
    lb = _lb()
    import torch

    with pytest.raises(lb.LBError, match="hipSetDevice"):
        lb.Lattice(8, 8, 8, 0.8, device=torch.cuda.device_count() + 3)


def test_device_bytes_fit_and_oversize_fails_cleanly():
    """A lattice larger than the card is refused with LB_ENOMEM, and the
    library stays usable."""
    lb = _lb()
    import torch

    free, _ = torch.cuda.mem_get_info()
    n = 1600  # 4.1e9 sites: FP64 needs ~40 TB
    assert lb.device_bytes(n, n, n) > free
    with pytest.raises(lb.LBError):
        lb.Lattice(n, n, n, 0.8, device=0)
    with lb.Lattice(8, 8, 8, 0.8, device=0) as g:
        g.init_fields(workloads.minkowski(8, 8, 8))
        g.step(1)


@pytest.mark.parametrize("lattice,shape,collision,matter", [
    (19, (5, 7, 13), 0, False),
    (19, (4, 6, 9), 1, True),
    (9, (1, 11, 17), 0, False),
])
def test_checkpoint_resume_is_exact(lattice, shape, collision, matter):
    """Saving the distributions after 10 steps and resuming them in a new
    handle continues bit for bit like the uninterrupted run (host and device
    buffers)."""
    lb = _lb()
    import torch

    nz, ny, nx = shape
    u0 = workloads.random_state(nx, ny, nz, seed=91, amp=0.03)
    G = workloads.random_matter(nx, ny, nz, seed=92, amp=1e-3) if matter else None
    kw = dict(device=0, lattice=lattice, collision=collision)
    with lb.Lattice(nx, ny, nz, 0.8, **kw) as a:
        if matter:
            a.set_matter(G)
        a.init_fields(u0)
        a.step(10)
        saved = a.distributions()
        a.step(15)
        ua, fa = a.moments(), a.distributions()
    for on_device in (False, True):
        with lb.Lattice(nx, ny, nz, 0.8, **kw) as b:
            if matter:
                b.set_matter(G)
            b.set_distributions(torch.from_numpy(saved).cuda() if on_device else saved)
            assert b.steps_done == 0
            b.step(15)
            assert np.array_equal(b.moments(), ua) and np.array_equal(b.distributions(), fa)


def test_checkpoint_resume_fp32():
    lb = _lb()
    u0 = workloads.random_state(13, 7, 5, seed=93, amp=0.03)
    with lb.Lattice(13, 7, 5, 0.8, precision=lb.FP32_DEV, device=0) as a:
        a.init_fields(u0)
        a.step(10)
        saved = a.distributions()
        a.step(15)
        ua = a.moments()
    with lb.Lattice(13, 7, 5, 0.8, precision=lb.FP32_DEV, device=0) as b:
        b.set_distributions(saved)
        b.step(15)
        ub = b.moments()
    assert np.abs(ub - ua).max() <= 1e-12


def test_check_finite_reports_the_blow_up():
    """The 1D gauge wave at tau = 0.55 goes non-finite after ~120 steps (the
    scheme's grid-scale instability); the check reports it, the run before it
    is finite."""
    lb = _lb()
    with lb.Lattice(100, 1, 1, 0.55, device=0) as g:
        g.init_fields(workloads.gauge_wave_x(100, 1, 1, 0.01, 100.0))
        g.step(50)
        assert g.check_finite()
        g.step(350)
        assert not g.check_finite()
        assert not np.all(np.isfinite(g.moments()))


class _Counting:
    """A DeviceAllocator over torch's caching allocator that counts calls and
    can be told to fail from its n-th allocation on."""

    def __init__(self, fail_from=None):
        from paper_1505_02037_amd import lb

        base = lb.TorchAllocator(0)
        outer = self

        class A(lb.DeviceAllocator):
            def alloc(self, nbytes):
                if outer.fail_from is not None and outer.allocs >= outer.fail_from:
                    return None
                outer.allocs += 1
                p = base.alloc(nbytes)
                outer.live[p] = nbytes
                return p

            def free(self, ptr):
                outer.frees += 1
                del outer.live[ptr]
                base.free(ptr)

        self.fail_from = fail_from
        self.allocs = self.frees = 0
        self.live = {}
        self.allocator = A()


def test_torch_allocator_serves_the_handle():
    """With the allocator hooks routed to torch's caching allocator the
    handle's buffers count in torch's accounting, go back to it on close, and
    the evolution is the default allocator's bit for bit."""
    lb = _lb()
    import torch

    u0 = workloads.random_state(13, 7, 5, seed=41)
    res = []
    for alloc in (None, "torch"):
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated(0)
        with lb.Lattice(13, 7, 5, 0.8, device=0, allocator=alloc) as g:
            held = torch.cuda.memory_allocated(0) - before
            if alloc == "torch":
                assert held >= lb.device_bytes(13, 7, 5)
            else:
                assert held == 0
            g.init_fields(u0)
            g.step(6)
            res.append((g.moments(), g.distributions()))
        assert torch.cuda.memory_allocated(0) == before
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_allocator_failure_is_enomem_and_releases_everything():
    lb = _lb()
    for fail_from in (0, 1, 3):
        c = _Counting(fail_from)
        with pytest.raises(lb.LBError, match="out of device memory"):
            lb.Lattice(8, 8, 8, 0.8, device=0, allocator=c.allocator)
        assert c.allocs == fail_from and c.frees == c.allocs and not c.live
    # per-site matter takes one more buffer from the same allocator
    c = _Counting()
    with lb.Lattice(6, 5, 4, 0.8, device=0, allocator=c.allocator) as g:
        n0 = c.allocs
        g.init_fields(workloads.minkowski(6, 5, 4))
        g.set_matter(workloads.random_matter(6, 5, 4, seed=3))
        g.step(2)
        assert c.allocs == n0 + 1
    assert c.frees == c.allocs and not c.live
