"""The wave configurations run on the GPU, as reports.

Each experiment prints one JSON object.  Errors are measured on the device
(lb_error_norms) against the analytic gauge wave, and, for the FP32 form,
against the FP64 step run alongside (the FP64 step equals the CPU oracle bit
for bit, as the parity tests show).

  c1   1D gauge wave: 100 sites, A = 0.01, d = 100, tau = 0.6, 10 crossings
  c2   3D x-wave: 128^3, A = 0.1, d = 128, tau in {0.55, 0.6, 1.0}, 20 crossings
  c2s  resolution series 32^3 / 64^3 / 128^3 at constant numerical diffusivity
  c3   256^3 (1,1,0) wave, A = 0.1, tau = 0.6, FP64 and FP32, 10 crossings
  c5   largest FP32 run that fits the card: x-wave A = 0.05 plus seeded
       Gaussian noise (sigma 1e-6) on the lapse, tau = 0.6, 1000 steps
  lin  linear (gravitational) wave at the paper's setup: 800 sites per
       wavelength, A = 1e-5, tau = 4.5, geodesic slicing, D3Q19
  gw   gauge wave at the paper's setup: 800 sites, A = 1e-3, tau = 4.5
  q9   D2Q9: the paper's gauge wave on its lattice, and 4096^2 throughput
  reg  life-times of BGK and of the regularized collision (declared variant)
  c3r  c3 with the regularized collision

Error measures (per field, group-scaled): max |u - ref| over the lattice,
divided by the max-norm of the field's tensor in ref (alpha alone, gamma, K
and V together); the life-time is the first checked step at which the
deviation-relative error of gamma_xx, max |g_xx - g_xx,ref| / max |g_xx,ref - 1|,
exceeds 10 %.

    python -m paper_1505_02037_amd.experiments c1 [c2 c2s c3 c5]
"""

from __future__ import annotations

import json
import math
import sys
import time

import numpy as np

from . import lb


def _torch():
    import torch

    assert torch.cuda.is_available(), "experiments need the GPU"
    torch.cuda.set_device(0)
    return torch


def _x_wave_dev(torch, n, nyz, A, d, t):
    import workloads

    return torch.from_numpy(workloads.gauge_wave_x(n, 1, 1, A, d, t=t)).cuda().expand(16, nyz[1], nyz[0], n).contiguous()


def _diag_dev(torch, n, nz, A, t):
    import workloads

    return torch.from_numpy(workloads.gauge_wave_diag(n, 1, A, t=t)).cuda().expand(16, nz, n, n).contiguous()


def _group_rel(norms, key="max_abs"):
    m = norms["ref_max"]
    scale = np.empty(16)
    scale[0] = m[0]
    scale[1:7] = m[1:7].max()
    scale[7:16] = max(m[7:16].max(), 1e-300)
    return norms[key] / scale


def _summary(norms):
    rel = _group_rel(norms)
    rl2 = _group_rel(norms, "l2")
    return {"alpha": float(rel[0]), "gamma": float(rel[1:7].max()), "K": float(rel[7:13].max()),
            "V": float(rel[13:16].max()), "l2_alpha": float(rl2[0]), "l2_gamma": float(rl2[1:7].max()),
            "l2_K": float(rl2[7:13].max())}


def _gxx_dev_rel(g, ref_dev):
    """deviation-relative error of gamma_xx against ref (device tensors)."""
    u = g.moments(ref_dev.new_empty(ref_dev.shape))
    num = (u[1] - ref_dev[1]).abs().max().item()
    den = (ref_dev[1] - 1.0).abs().max().item()
    return num / den if den > 0 else float("nan")


def c1():
    """1D gauge wave, ten crossings, errors each crossing, life-time."""
    torch = _torch()
    n, A, d, tau = 100, 0.01, 100.0, 0.6
    out = {"experiment": "c1 1D gauge wave", "N": n, "A": A, "d": d, "tau": tau, "crossings": []}
    with lb.Lattice(n, 1, 1, tau, device=0) as g:
        g.init_fields(_x_wave_dev(torch, n, (1, 1), A, d, 0.0))
        life = None
        for step in range(0, 1001, 10):
            if step:
                g.step(10)
            ref = _x_wave_dev(torch, n, (1, 1), A, d, float(step))
            if life is None:
                e = _gxx_dev_rel(g, ref)
                if not (e <= 0.10):
                    life = step
            if step % 100 == 0:
                out["crossings"].append({"step": step, **_summary(g.error_norms(ref))})
        out["lifetime_steps"] = life
    return out


def c2():
    """3D x-wave at 128^3, three relaxation times, 20 crossings."""
    torch = _torch()
    n, A = 128, 0.1
    out = {"experiment": "c2 3D x-wave 128^3", "A": A, "d": n, "runs": []}
    for tau in (0.55, 0.6, 1.0):
        run = {"tau": tau, "crossings": []}
        t0 = time.perf_counter()
        with lb.Lattice(n, n, n, tau, device=0) as g:
            g.init_fields(_x_wave_dev(torch, n, (n, n), A, float(n), 0.0))
            life = None
            for step in range(0, 20 * n + 1, 32):
                if step:
                    g.step(32)
                if life is None or step % n == 0:
                    ref = _x_wave_dev(torch, n, (n, n), A, float(n), float(step))
                    if life is None:
                        e = _gxx_dev_rel(g, ref)
                        if not (e <= 0.10):
                            life = step
                    if step % n == 0:
                        run["crossings"].append({"step": step, **_summary(g.error_norms(ref))})
            run["lifetime_steps"] = life
        run["wall_s"] = time.perf_counter() - t0
        out["runs"].append(run)
    return out


def c2s():
    """Resolution series at constant numerical diffusivity
    eta = (tau - 1/2) c_s^2 dx (physical units, dt = dx = 1/N, d = 1):
    tau_N = 1/2 + (tau_128 - 1/2) N / 128.  Error of gamma_xx at a fixed step
    count (400, the paper's protocol) and at a fixed physical time (one
    crossing, N steps); order = log2 of successive error ratios."""
    torch = _torch()
    A = 0.1
    out = {"experiment": "c2s resolution series at constant eta", "A": A, "series": []}
    for tau128 in (1.0, 2.0):
        ser = {"tau_128": tau128, "eta_phys": (tau128 - 0.5) / 3.0 / 128.0, "points": []}
        for n in (32, 64, 128):
            tau = 0.5 + (tau128 - 0.5) * n / 128.0
            pt = {"N": n, "tau": tau}
            with lb.Lattice(n, n, n, tau, device=0) as g:
                g.init_fields(_x_wave_dev(torch, n, (n, n), A, float(n), 0.0))
                done = 0
                for tag, step in (("crossing", n), ("step400", 400)):
                    g.step(step - done)
                    done = step
                    pt[tag] = _gxx_dev_rel(g, _x_wave_dev(torch, n, (n, n), A, float(n), float(step)))
            ser["points"].append(pt)
        for tag in ("crossing", "step400"):
            e = [p[tag] for p in ser["points"]]
            ser[f"order_{tag}"] = [math.log2(e[i] / e[i + 1]) if e[i + 1] > 0 else None for i in range(2)]
        out["series"].append(ser)
    return out


def c3(collision=lb.COLLISION_BGK):
    """256^3 diagonal wave, FP64 and FP32 side by side, ten crossings."""
    torch = _torch()
    n, A, tau = 256, 0.1, 0.6
    cross = n / math.sqrt(2.0)
    steps = int(round(10 * cross))
    checks = sorted(set([1, 2, 5, 10, 20, 50, 100, 150, 200, 300, 400, 500, 600, 700]
                        + [int(round(k * cross)) for k in range(1, 11)]))
    out = {"experiment": "c3 256^3 diagonal wave", "A": A, "tau": tau, "steps": steps,
           "collision": "regularized" if collision else "bgk", "checks": []}
    u0 = _diag_dev(torch, n, n, A, 0.0)
    g64 = lb.Lattice(n, n, n, tau, precision=lb.FP64, device=0, collision=collision)
    g32 = lb.Lattice(n, n, n, tau, precision=lb.FP32_DEV, device=0, collision=collision)
    g64.init_fields(u0)
    g32.init_fields(u0)
    del u0
    u64 = torch.empty((16, n, n, n), dtype=torch.float64, device="cuda")
    done, life64, life32, horizon32 = 0, None, None, None
    for c in checks:
        if c > steps:
            break
        g64.step(c - done)
        g32.step(c - done)
        done = c
        ref = _diag_dev(torch, n, n, A, float(c))
        e64 = _summary(g64.error_norms(ref))
        e32 = _summary(g32.error_norms(ref))
        g64.moments(u64)
        d32 = _summary(g32.error_norms(u64))  # FP32 form against the FP64 step
        worst = max(d32["alpha"], d32["gamma"], d32["K"], d32["V"])
        if horizon32 is None and not (worst <= 1e-5):
            horizon32 = c
        if life64 is None and not (_gxx_dev_rel(g64, ref) <= 0.1):
            life64 = c
        if life32 is None and not (_gxx_dev_rel(g32, ref) <= 0.1):
            life32 = c
        out["checks"].append({"step": c, "fp64_vs_analytic": e64, "fp32_vs_analytic": e32, "fp32_vs_fp64": d32})
        print(json.dumps(out["checks"][-1]), flush=True)
    out.update({"lifetime_fp64_steps": life64, "lifetime_fp32_steps": life32,
                "fp32_within_1e-5_until_step_before": horizon32})
    g64.close()
    g32.close()
    return out


def c5(margin_gib: float = 3.0):
    """Largest cubic FP32 run that fits: two distribution buffers plus the
    FP64 per-site scratch of lb_device_bytes, within the free device memory
    less a margin."""
    torch = _torch()
    import workloads

    free, total = torch.cuda.mem_get_info()
    budget = free - margin_gib * (1 << 30)
    e = 256
    while lb.device_bytes(e + 1, e + 1, e + 1, precision=lb.FP32_DEV) <= budget:
        e += 1
    nbytes = lb.device_bytes(e, e, e, precision=lb.FP32_DEV)
    A, tau, sigma, seed = 0.05, 0.6, 1e-6, 1505
    # host fields: x-wave plus lapse noise (seeded PCG64), staged through the library
    u0 = np.broadcast_to(workloads.gauge_wave_x(e, 1, 1, A, float(e)), (16, e, e, e)).copy()
    rng = np.random.Generator(np.random.PCG64(seed))
    for z in range(e):
        u0[0, z] += sigma * rng.standard_normal((e, e))
    out = {"experiment": "c5 largest FP32 run", "edge": e, "sites": e ** 3, "device_bytes": nbytes,
           "device_total_bytes": total, "A": A,
           "tau": tau, "noise_sigma": sigma, "seed": seed}
    g = lb.Lattice(e, e, e, tau, precision=lb.FP32_DEV, device=0)
    g.init_fields(u0)
    del u0
    g.step(2)
    torch.cuda.synchronize()
    g.set_timing(True)
    t0 = time.perf_counter()
    g.step(1000)
    wall = time.perf_counter() - t0
    kt = g.kernel_times()
    out.update({"steps": 1000, "wall_s": wall, "ms_per_step": 1000 * wall / 1000,
                "field_site_updates_per_s": 16 * e ** 3 * 1000 / wall, "kernel_ms": kt,
                "algorithmic_GBps": 2432 * e ** 3 / (sum(kt.values()) * 1e-3) / 1e9})
    g.close()
    return out


def _paper_wave(name, make, field, slicing, A, tau=4.5, n=800, steps=3000, lattice=lb.D3Q19):
    """Error of `field` against its analytic wave every 100 steps and the
    step at which its deviation-relative error first exceeds 10 %."""
    torch = _torch()
    out = {"experiment": name, "N": n, "A": A, "tau": tau, "lattice": lattice, "checks": []}
    with lb.Lattice(n, 1, 1, tau, slicing=slicing, device=0, lattice=lattice) as g:
        g.init_fields(make(n, 1, 1, A, float(n)))
        life = None
        u = torch.empty((16, 1, 1, n), dtype=torch.float64, device="cuda")
        rest = 1.0 if field in (0, 1, 4, 6) else 0.0
        for step in range(0, steps + 1, 100):
            if step:
                g.step(100)
            ref = torch.from_numpy(make(n, 1, 1, A, float(n), t=float(step))).cuda()
            g.moments(u)
            dev = ((u[field] - ref[field]).abs().max() / (ref[field] - rest).abs().max()).item()
            val = _summary(g.error_norms(ref))
            out["checks"].append({"step": step, "dev_rel": dev, **val})
            if life is None and not (dev <= 0.10):
                life = step
        out["lifetime_steps"] = life
    return out


def lin():
    import workloads

    return _paper_wave("lin linear wave, paper setup", workloads.linear_wave_x, 4, lb.GEODESIC, 1e-5)


def gw():
    import workloads

    return _paper_wave("gw gauge wave, paper setup", workloads.gauge_wave_x, 1, lb.HARMONIC, 1e-3)


def q9():
    """D2Q9: the paper's gauge wave on its own lattice, and the throughput of
    the D2Q9 step on a 4096 x 4096 lattice ((1,1,0) wave, tau = 0.6) in both
    storage forms."""
    import workloads

    torch = _torch()
    out = {"experiment": "q9 D2Q9", "paper_gauge_wave": _paper_wave(
        "gauge wave, paper setup, D2Q9", workloads.gauge_wave_x, 1, lb.HARMONIC, 1e-3, lattice=lb.D2Q9)}
    out["paper_gauge_wave"].pop("checks")
    n, tau, steps = 4096, 0.6, 20
    u0 = torch.from_numpy(workloads.gauge_wave_diag(n, 1, 0.1)).cuda()
    for form, prec, bps in (("fp64", lb.FP64, 2 * 16 * 9 * 8), ("fp32", lb.FP32_DEV, 2 * 16 * 9 * 4)):
        with lb.Lattice(n, n, 1, tau, precision=prec, device=0, lattice=lb.D2Q9) as g:
            g.init_fields(u0)
            g.step(3)
            torch.cuda.synchronize()
            g.set_timing(True)
            t0 = time.perf_counter()
            g.step(steps)
            wall = time.perf_counter() - t0
            kt = g.kernel_times()
        out[form] = {"lattice": [n, n, 1], "steps": steps, "ms_per_step": 1000 * wall / steps,
                     "field_site_updates_per_s": 16 * n * n * steps / wall, "kernel_ms": kt,
                     "algorithmic_GBps": bps * n * n / (sum(kt.values()) * 1e-3) / 1e9}
    return out


def _life(torch, make_lattice, ref_at, steps, every):
    """First checked step at which gamma_xx deviates from the wave by more
    than 10 % of its amplitude (or the state is non-finite), and the step at
    which it first turns non-finite."""
    with make_lattice() as g:
        g.init_fields(ref_at(0.0))
        life, blow, n = None, None, 0
        while n < steps:
            g.step(every)
            n += every
            ref = ref_at(float(n))
            u = g.moments(ref.new_empty(ref.shape))
            finite = bool(torch.isfinite(u).all().item())
            if not finite:
                blow = n
                life = life or n
                break
            e = (u[1] - ref[1]).abs().max().item() / (ref[1] - 1.0).abs().max().item()
            if life is None and e > 0.10:
                life = n
        return life, blow


def reg():
    """Life-times of the BGK step and of the regularized collision (a
    declared variant) on the gauge-wave configurations, FP64."""
    torch = _torch()
    out = {"experiment": "reg BGK vs regularized life-times", "runs": []}
    cases = [
        ("1D x-wave 100, A=0.01", 0.6, lambda t: _x_wave_dev(torch, 100, (1, 1), 0.01, 100.0, t), (100, 1, 1), 3000, 10),
        ("1D x-wave 100, A=0.01", 0.55, lambda t: _x_wave_dev(torch, 100, (1, 1), 0.01, 100.0, t), (100, 1, 1), 3000, 10),
        ("3D x-wave 128^3, A=0.1", 0.55, lambda t: _x_wave_dev(torch, 128, (128, 128), 0.1, 128.0, t), (128, 128, 128), 2560, 16),
        ("3D x-wave 128^3, A=0.1", 0.6, lambda t: _x_wave_dev(torch, 128, (128, 128), 0.1, 128.0, t), (128, 128, 128), 2560, 16),
        ("3D x-wave 128^3, A=0.1", 1.0, lambda t: _x_wave_dev(torch, 128, (128, 128), 0.1, 128.0, t), (128, 128, 128), 2560, 16),
        ("256^3 (1,1,0) wave, A=0.1", 0.6, lambda t: _diag_dev(torch, 256, 256, 0.1, t), (256, 256, 256), 1810, 10),
    ]
    for name, tau, ref_at, shape, steps, every in cases:
        row = {"case": name, "tau": tau, "steps": steps}
        for coll, key in ((lb.COLLISION_BGK, "bgk"), (lb.COLLISION_REGULARIZED, "regularized")):
            t0 = time.perf_counter()
            life, blow = _life(torch, lambda: lb.Lattice(*shape, tau, device=0, collision=coll), ref_at, steps, every)
            row[key] = {"lifetime_steps": life, "nonfinite_at": blow, "wall_s": time.perf_counter() - t0}
        print(json.dumps(row), flush=True)
        out["runs"].append(row)
    return out


def main(argv=None) -> int:
    which = (argv if argv is not None else sys.argv[1:]) or ["c1"]
    for w in which:
        res = {"c1": c1, "c2": c2, "c2s": c2s, "c3": c3, "c5": c5, "lin": lin, "gw": gw, "q9": q9, "reg": reg,
               "c3r": lambda: c3(lb.COLLISION_REGULARIZED)}[w]()
        print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
