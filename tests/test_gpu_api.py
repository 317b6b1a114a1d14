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

    with pytest.raises(lb.LBError):
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
