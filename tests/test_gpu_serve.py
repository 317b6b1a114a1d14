"""GPU: the served form (continuous batching, include/lb_serve.h).

Each request's result must be the same alone and in the mix, bit for bit:
the batched kernels run the same per-site step as the single-lattice path, and
requests never share memory.  Also: exact per-request step counts when the
graph's step count does not divide them, admission never exceeds the HBM
budget, a request that goes non-finite is reported FAILED without touching
the others, and the trace driver reports time to solution and throughput.
"""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch

    assert torch.cuda.is_available(), "GPU test run without a GPU"


def _alone(u0, tau, steps, precision):
    from paper_1505_02037_amd import lb

    nz, ny, nx = u0.shape[1:]
    with lb.Lattice(nx, ny, nz, tau, precision=precision, device=0) as g:
        g.init_fields(u0)
        g.step(steps)
        return g.moments()


REQS = [
    # (shape nz, ny, nx), tau, steps, seed
    ((6, 7, 13), 0.7, 11, 1),
    ((16, 16, 16), 0.9, 23, 2),
    ((3, 20, 33), 0.62, 5, 3),
    ((1, 1, 40), 1.1, 17, 4),
    ((9, 8, 7), 0.8, 0, 5),
]


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_alone_equals_mix_bitwise(form):
    _need_gpu()
    from paper_1505_02037_amd import lb, serve

    prec = lb.FP64 if form == "fp64" else lb.FP32_DEV
    print(f"[serve] alone vs mix, {form}", flush=True)
    inputs = [workloads.random_state(s[2], s[1], s[0], seed=seed, amp=0.05) for s, _, _, seed in REQS]
    alone = [_alone(u0, tau, steps, prec) for u0, (_, tau, steps, _) in zip(inputs, REQS)]
    with serve.Server(1 << 30, prec, max_resident=8, steps_per_launch=4, device=0) as srv:
        ids = [srv.submit(u0, tau, steps) for u0, (_, tau, steps, _) in zip(inputs, REQS)]
        for _ in range(100):
            if srv.advance() == 0:
                break
        for rid, ref, (_, _, steps, _) in zip(ids, alone, REQS):
            inf = srv.info(rid)
            assert inf.state == serve.DONE and inf.steps_done == steps
            assert np.array_equal(srv.result(rid), ref)
        st = srv.stats()
    assert st["completed"] == len(REQS) and st["resident"] == 0 and st["arena_in_use"] == 0


def test_largest_trace_request_alongside_a_small_one():
    """The trace's largest request size (192^3, random state) resident
    together with a small request: both equal their solo runs bit for bit
    (the work list spans ~27600 blocks of the large request)."""
    _need_gpu()
    from paper_1505_02037_amd import lb, serve

    print("[serve] 192^3 request beside a small one", flush=True)
    big = workloads.random_state(192, 192, 192, seed=192, amp=0.05)
    small = workloads.random_state(13, 7, 5, seed=193, amp=0.05)
    ref_big = _alone(big, 0.8, 3, lb.FP64)
    ref_small = _alone(small, 0.7, 7, lb.FP64)
    with serve.Server(1 << 30, lb.FP64, device=0) as probe:
        need = probe.request_bytes(192, 192, 192) + probe.request_bytes(13, 7, 5)
    with serve.Server(need + (1 << 24), lb.FP64, max_resident=4, steps_per_launch=2, device=0) as srv:
        ib = srv.submit(big, 0.8, 3)
        i_s = srv.submit(small, 0.7, 7)
        for _ in range(20):
            if srv.advance() == 0:
                break
        assert np.array_equal(srv.result(ib), ref_big)
        assert np.array_equal(srv.result(i_s), ref_small)


def test_budget_limits_residency():
    """A budget that holds one large request at a time: requests are admitted
    as memory frees up, all finish, and the arena never exceeds the budget."""
    _need_gpu()
    from paper_1505_02037_amd import lb, serve

    print("[serve] small budget", flush=True)
    shapes = [(12, 12, 12), (10, 11, 12), (12, 12, 12), (5, 6, 7)]
    inputs = [workloads.random_state(s[2], s[1], s[0], seed=10 + i) for i, s in enumerate(shapes)]
    with serve.Server(1 << 30, lb.FP64, device=0) as probe:
        need = probe.request_bytes(12, 12, 12)
    budget = int(need * 1.5)
    alone = [_alone(u0, 0.75, 9, lb.FP64) for u0 in inputs]
    with serve.Server(budget, lb.FP64, max_resident=8, steps_per_launch=2, device=0) as srv:
        ids = [srv.submit(u0, 0.75, 9) for u0 in inputs]
        peak_res = 0
        for _ in range(200):
            active = srv.advance()
            peak_res = max(peak_res, srv.stats()["resident"])
            if active == 0:
                break
        st = srv.stats()
        assert st["arena_peak"] <= st["arena_bytes"] <= budget
        for rid, ref in zip(ids, alone):
            assert np.array_equal(srv.result(rid), ref)
    assert st["completed"] == 4


def test_nonfinite_request_is_failed_and_isolated():
    _need_gpu()
    from paper_1505_02037_amd import lb, serve

    print("[serve] non-finite request", flush=True)
    bad = workloads.random_state(16, 16, 16, seed=21, amp=0.25)
    good = workloads.gauge_wave_x(20, 4, 4, 0.05, 20)
    ref = _alone(good, 0.9, 150, lb.FP64)
    with serve.Server(1 << 30, lb.FP64, steps_per_launch=16, device=0) as srv:
        ib = srv.submit(bad, 0.51, 400)
        ig = srv.submit(good, 0.9, 150)
        while srv.advance():
            pass
        assert srv.info(ib).state == serve.FAILED
        assert srv.info(ig).state == serve.DONE
        assert np.array_equal(srv.result(ig), ref)
        assert not np.isfinite(srv.result(ib)).all()


def test_bad_device_is_an_error_not_a_fault():
    _need_gpu()
    import torch
    from paper_1505_02037_amd import lb, serve

    with pytest.raises(lb.LBError, match="hipSetDevice"):
        serve.Server(1 << 20, lb.FP64, device=torch.cuda.device_count() + 3)
    with serve.Server(1 << 20, lb.FP64, device=0) as srv:  # still usable afterwards
        assert srv.stats()["resident"] == 0


def test_trace_driver_reports_tts():
    _need_gpu()
    from paper_1505_02037_amd import lb, serve

    print("[serve] small trace", flush=True)
    reqs = workloads.request_trace(seed=7, rate_hz=50.0, count=8, nmin=12, nmax=32, smin=10, smax=60)
    rep, res = serve.run_trace(reqs, lb.FP64, budget_bytes=4 << 30, steps_per_launch=4, keep_results=True)
    assert rep["completed"] + rep["failed_nonfinite"] == 8
    assert 0 < rep["tts_p50_s"] <= rep["tts_p99_s"] <= rep["wall_s"]
    expect = sum(r.n ** 3 * r.steps for r in reqs)
    assert rep["site_updates"] == expect
    # one request checked against its own single-lattice run
    r = reqs[3]
    ref = _alone(workloads.gauge_wave_x(r.n, r.n, r.n, r.amp, float(r.n)), r.tau, r.steps, lb.FP64)
    assert np.array_equal(res[r.rid], ref, equal_nan=True)
