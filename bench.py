"""Throughput of the Bona-Masso lattice Boltzmann step on one MI355X.

Workload: the 256^3 periodic lattice with the gauge wave along the (1,1,0)
diagonal, A = 0.1, tau = 0.6, harmonic slicing, FP64 storage and arithmetic.
One "step" is one lattice Boltzmann time
step over the whole lattice (moments, lapse/metric half source, derivative
stencil, geometry and sources, flux, equilibria, BGK relaxation with source,
pull streaming).  Inputs are resident in HBM before timing starts.

Prints one JSON line with the throughput in field-site updates per second
(16 fields per site), the roofline of the step against HBM bandwidth
(algorithmic bytes: every distribution read once and written once, 16 x 19 x
8 B each way per site), and the CPU oracle timed on a bounded sample of the
same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--form fp64|fp32]
                    [--path split|fused] [--collision bgk|regularized] [--no-cpu]
    python bench.py --cpu-table   (the oracle alone: single-threaded and all host threads)
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FIELDS, Q = 16, 19
# read + write every distribution once, per site update
ALG_BYTES_PER_SITE = {"fp64": 2 * FIELDS * Q * 8, "fp32": 2 * FIELDS * Q * 4}


# the device sources the timed step kernels are compiled from (host-side
# launch code is not part of a kernel)
STEP_SOURCES = ("lb_device.h", "lb_fp32.hip", "lb_fp64.hip", "lb_kernels.h", "lb_site.h", "lb_step.h")


def _code_only(text: str) -> str:
    """Source text without comments and blank space (the device sources hold
    no string literals), so that editing a comment keeps the hash."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    """Hash of the code of the sources the timed step kernels are built from,
    and of the plane padding the host sets (it moves the kernels' addresses)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1505_02037_amd", "csrc")
    for name in STEP_SOURCES:
        h.update(_code_only(open(os.path.join(csrc, name)).read()).encode())
    pad = re.search(r"constexpr size_t kPlanePad = (\d+);", open(os.path.join(csrc, "lb_api.hip")).read())
    h.update(f"plane pad {pad.group(1) if pad else 'none'}".encode())
    return h.hexdigest()[:16]


def measured_traffic(nsite: int, form: str):
    """HBM bytes per step from the committed counter summary, if it was taken
    on the current kernels (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{form}_step.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d["bytes_per_site_per_step"] * nsite


def cpu_baseline(n: int, tau: float, target_s: float = 15.0) -> dict:
    """The oracle (plain FP64 C, OpenMP over sites) on a bounded sample of the
    same workload: the (1,1,0) wave on n x n x 8 sites."""
    import oracle
    import workloads

    nz = 8
    u0 = workloads.gauge_wave_diag(n, nz, 0.1)
    o = oracle.Oracle(n, n, nz, tau)
    o.init_fields(u0)
    t0 = time.perf_counter()
    o.step(1)
    dt1 = time.perf_counter() - t0
    steps = max(1, min(2000, int(target_s / max(dt1, 1e-6))))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    sites = n * n * nz
    return {
        "value": FIELDS * sites * steps / dt,
        "unit": "field-site updates/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"(1,1,0) gauge wave A=0.1 tau={tau} on {n}x{n}x{nz} sites, {steps} steps, {dt:.1f} s",
    }


CPU_CASES = {
    # name: (description, nx, ny, nz, steps at all threads, steps single-threaded, workload)
    "c1": ("1D x-wave, 100 sites, A=0.01, tau=0.6", 100, 1, 1, 1000, 1000, "x"),
    "64cubed": ("3D x-wave 64^3, A=0.1, tau=0.6", 64, 64, 64, 20, 4, "x"),
    "128cubed": ("3D x-wave 128^3, A=0.1, tau=0.6", 128, 128, 128, 10, 1, "x"),
}


def cpu_case(name: str, single: bool) -> dict:
    """The oracle on one CPU case (run in a child process whose OpenMP
    thread count is set by its environment)."""
    import oracle
    import workloads

    desc, nx, ny, nz, steps_all, steps_one, _ = CPU_CASES[name]
    steps = steps_one if single else steps_all
    A = 0.01 if name == "c1" else 0.1
    o = oracle.Oracle(nx, ny, nz, 0.6)
    o.init_fields(workloads.gauge_wave_x(nx, ny, nz, A, float(nx)))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    n = nx * ny * nz
    return {"case": desc, "threads": oracle.num_threads(), "steps": steps, "seconds": dt,
            "site_updates_per_s": n * steps / dt, "field_site_updates_per_s": FIELDS * n * steps / dt}


def cpu_table() -> int:
    """The oracle timed single-threaded and on all host threads (one child
    process per measurement, OMP_NUM_THREADS set for it)."""
    import subprocess

    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    allt = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    rows = []
    for name in CPU_CASES:
        for threads in ("1", allt):
            env = dict(os.environ, OMP_NUM_THREADS=threads)
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-case", name,
                                "--single" if threads == "1" else "--all"],
                               env=env, capture_output=True, text=True, check=True)
            rows.append(json.loads(r.stdout.strip().splitlines()[-1]))
            print(json.dumps(rows[-1]), flush=True)
    print(json.dumps({"cpu_model": model, "logical_cpus": os.cpu_count(), "omp_all_threads": int(allt),
                      "kind": "oracle", "rows": rows}), flush=True)
    return 0


def main() -> int:
    if "--cpu-case" in sys.argv:
        name = sys.argv[sys.argv.index("--cpu-case") + 1]
        print(json.dumps(cpu_case(name, "--single" in sys.argv)), flush=True)
        return 0
    if "--cpu-table" in sys.argv:
        return cpu_table()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--tau", type=float, default=0.6)
    ap.add_argument("--form", choices=("fp64", "fp32"), default="fp64",
                    help="fp64: plain FP64 step; fp32: FP32-deviation storage and relaxation")
    ap.add_argument("--path", choices=("split", "fused"), default="split",
                    help="split: two launches per step (the library's default); fused: one z-marching launch")
    ap.add_argument("--collision", choices=("bgk", "regularized"), default="bgk",
                    help="bgk: the paper's collision (the headline); regularized: the declared variant")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is described in the design notes, not built)"}))
        return 2

    import torch

    import workloads
    from paper_1505_02037_amd import lb

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 2
    torch.cuda.set_device(0)
    n, tau = args.n, args.tau
    nsite = n * n * n
    stream = torch.cuda.Stream()
    precision = lb.FP64 if args.form == "fp64" else lb.FP32_DEV
    path = lb.PATH_SPLIT if args.path == "split" else lb.PATH_FUSED
    collision = lb.COLLISION_BGK if args.collision == "bgk" else lb.COLLISION_REGULARIZED
    g = lb.Lattice(n, n, n, tau, precision=precision, device=0, stream=stream.cuda_stream, path=path,
                   collision=collision)
    with torch.cuda.stream(stream):
        u0 = torch.from_numpy(workloads.gauge_wave_diag(n, 1, 0.1)).cuda().expand(16, n, n, n).contiguous()
    stream.synchronize()
    g.init_fields(u0)
    del u0
    g.step(args.warmup)
    stream.synchronize()

    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)          # timed with HIP events per kernel on the handle's stream
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ktimes = g.kernel_times()
    g.close()

    ms_step = 1000.0 * wall / args.steps
    value = FIELDS * nsite * args.steps / wall
    step_kernel_ms = sum(ktimes.values())
    alg_bytes = ALG_BYTES_PER_SITE[args.form] * nsite
    achieved = alg_bytes / (step_kernel_ms * 1e-3) / 1e9
    # the counters were taken on the default launch at 256^3
    traffic = (measured_traffic(nsite, args.form)
               if (args.path, args.collision, n) == ("split", "bgk", 256) else None)
    line = {
        "metric": "field-site updates/s",
        "value": value,
        "unit": "field-site updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.form == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"3D gauge wave along (1,1,0), {n}^3 periodic, A=0.1, tau={tau}, harmonic slicing, "
                        + ("FP64 distributions" if args.form == "fp64" else
                           "FP32 deviation distributions (FP64 moments/geometry)")
                        + ", D3Q19, 16 Bona-Masso fields",
            "lattice": [n, n, n],
            "tau": tau,
            "form": args.form,
            "path": args.path,
            "collision": args.collision,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "+".join(ktimes.keys()),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_step": alg_bytes,
            "kernel_ms": ktimes,
        },
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(128, tau)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
