"""Binding of the serving C-ABI (include/lb_serve.h) and a trace replay.

run_trace replays a seeded Poisson trace of independent gauge-wave
evolutions in real time: each request is submitted when its arrival time has
passed, the server advances every resident request together one graph launch
at a time, and finished requests are retired.  It reports the time to
solution (completion minus arrival, host monotonic clock) at p50 and p99 and
the aggregate throughput in site and field-site updates per second.

    python -m paper_1505_02037_amd.serve [--count 24] [--form fp64|fp32] ...
"""

from __future__ import annotations

import argparse
import ctypes
import json
import sys
import time

import numpy as np

from . import lb

QUEUED, RUNNING, DONE, FAILED = 0, 1, 2, 3
EXPORTS = (
    "lb_server_create", "lb_server_request_bytes", "lb_server_submit", "lb_server_advance",
    "lb_server_info", "lb_server_result", "lb_server_get_stats", "lb_server_destroy",
)


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("precision", ctypes.c_int),
        ("max_resident", ctypes.c_int),
        ("steps_per_launch", ctypes.c_int),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class RequestInfo(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int),
        ("steps_done", ctypes.c_longlong),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("graph_launches", ctypes.c_longlong),
        ("site_updates", ctypes.c_longlong),
        ("completed", ctypes.c_longlong),
        ("failed", ctypes.c_longlong),
        ("resident", ctypes.c_int),
        ("queued", ctypes.c_int),
        ("arena_bytes", ctypes.c_size_t),
        ("arena_in_use", ctypes.c_size_t),
        ("arena_peak", ctypes.c_size_t),
    ]


def _lib():
    lib = lb.load_library()
    if getattr(lib, "_serve_ready", False):
        return lib
    P = ctypes.c_void_p
    lib.lb_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]
    lib.lb_server_request_bytes.argtypes = [P, ctypes.POINTER(lb.LBConfig)]
    lib.lb_server_request_bytes.restype = ctypes.c_size_t
    lib.lb_server_submit.argtypes = [P, ctypes.POINTER(lb.LBConfig), P, ctypes.c_longlong,
                                     ctypes.POINTER(ctypes.c_ulonglong)]
    lib.lb_server_advance.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
    lib.lb_server_info.argtypes = [P, ctypes.c_ulonglong, ctypes.POINTER(RequestInfo)]
    lib.lb_server_result.argtypes = [P, ctypes.c_ulonglong, P]
    lib.lb_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.lb_server_destroy.argtypes = [P]
    lib.lb_server_destroy.restype = None
    lib._serve_ready = True
    return lib


class Server:
    """Continuous-batching server of independent evolutions (one GPU)."""

    def __init__(self, budget_bytes: int, precision: int = lb.FP64, max_resident: int = 64,
                 steps_per_launch: int = 8, device: int = -1):
        lib = _lib()
        self._lib = lib
        cfg = ServerConfig(int(budget_bytes), int(precision), int(max_resident), int(steps_per_launch),
                           int(device), None)
        h = ctypes.c_void_p()
        lb._check(lib.lb_server_create(ctypes.byref(cfg), ctypes.byref(h)), "lb_server_create")
        self._h = h
        self.shapes = {}

    def close(self):
        if self._h:
            self._lib.lb_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def request_bytes(self, nx, ny, nz, tau=0.6) -> int:
        cfg = lb.make_config(nx, ny, nz, tau)
        return int(self._lib.lb_server_request_bytes(self._h, ctypes.byref(cfg)))

    def submit(self, u0: np.ndarray, tau: float, nsteps: int, slicing: int = lb.HARMONIC) -> int:
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        nz, ny, nx = u0.shape[1:]
        cfg = lb.make_config(nx, ny, nz, tau, slicing)
        rid = ctypes.c_ulonglong()
        lb._check(self._lib.lb_server_submit(self._h, ctypes.byref(cfg), ctypes.c_void_p(u0.ctypes.data),
                                             int(nsteps), ctypes.byref(rid)), "lb_server_submit")
        self.shapes[rid.value] = (nz, ny, nx)
        return rid.value

    def advance(self) -> int:
        n = ctypes.c_int()
        lb._check(self._lib.lb_server_advance(self._h, ctypes.byref(n)), "lb_server_advance")
        return n.value

    def info(self, rid: int) -> RequestInfo:
        inf = RequestInfo()
        lb._check(self._lib.lb_server_info(self._h, rid, ctypes.byref(inf)), "lb_server_info")
        return inf

    def result(self, rid: int) -> np.ndarray:
        out = np.empty((16,) + self.shapes[rid], dtype=np.float64)
        lb._check(self._lib.lb_server_result(self._h, rid, ctypes.c_void_p(out.ctypes.data)), "lb_server_result")
        del self.shapes[rid]
        return out

    def stats(self) -> dict:
        st = ServerStats()
        lb._check(self._lib.lb_server_get_stats(self._h, ctypes.byref(st)), "lb_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}


def run_trace(requests, precision=lb.FP64, budget_bytes=200 << 30, max_resident=64,
              steps_per_launch=8, keep_results=False, log=None):
    """Replay `requests` (workloads.trace.Request) in real time; return a report."""
    import workloads

    srv = Server(budget_bytes, precision, max_resident, steps_per_launch)
    pending = sorted(requests, key=lambda r: r.arrival_s)
    ids, done, results = {}, {}, {}
    t0 = time.perf_counter()
    i = 0
    while i < len(pending) or len(done) < len(pending):
        now = time.perf_counter() - t0
        while i < len(pending) and pending[i].arrival_s <= now:
            r = pending[i]
            u0 = workloads.gauge_wave_x(r.n, r.n, r.n, r.amp, float(r.n))
            ids[srv.submit(u0, r.tau, r.steps)] = r
            i += 1
        active = srv.advance()
        for rid in list(ids):
            if rid in done:
                continue
            inf = srv.info(rid)
            if inf.state in (DONE, FAILED):
                done[rid] = (inf.state, inf.t_done - inf.t_submit)
                res = srv.result(rid)
                if keep_results:
                    results[ids[rid].rid] = res
                if log:
                    log(f"request {ids[rid].rid} N={ids[rid].n} steps={ids[rid].steps} "
                        f"{'done' if inf.state == DONE else 'FAILED'} tts={inf.t_done - inf.t_submit:.2f}s")
        if active == 0 and i < len(pending):
            time.sleep(max(0.0, min(0.05, pending[i].arrival_s - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    tts = np.array([v[1] for v in done.values()])
    report = {
        "requests": len(pending),
        "completed": int(st["completed"]),
        "failed_nonfinite": int(st["failed"]),
        "wall_s": wall,
        "tts_p50_s": float(np.percentile(tts, 50)),
        "tts_p99_s": float(np.percentile(tts, 99)),
        "site_updates": int(st["site_updates"]),
        "site_updates_per_s": st["site_updates"] / wall,
        "field_site_updates_per_s": 16 * st["site_updates"] / wall,
        "graph_launches": int(st["graph_launches"]),
        "arena_bytes": int(st["arena_bytes"]),
        "arena_peak_bytes": int(st["arena_peak"]),
    }
    return (report, results) if keep_results else report


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=24, help="first N arrivals of the trace")
    ap.add_argument("--seed", type=int, default=1505)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--form", choices=("fp64", "fp32"), default="fp64")
    ap.add_argument("--budget-gib", type=float, default=200.0)
    ap.add_argument("--max-resident", type=int, default=64)
    ap.add_argument("--steps-per-launch", type=int, default=8)
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args(argv)
    import workloads

    reqs = workloads.request_trace(seed=args.seed, rate_hz=args.rate, count=args.count)
    prec = lb.FP64 if args.form == "fp64" else lb.FP32_DEV
    rep = run_trace(reqs, prec, int(args.budget_gib * (1 << 30)), args.max_resident, args.steps_per_launch,
                    log=(lambda m: print(m, flush=True)) if args.verbose else None)
    rep.update({"form": args.form, "trace": {"seed": args.seed, "rate_hz": args.rate, "count": args.count,
                                             "N": "log-uniform [32,192]", "A": "U[1e-3,0.2]",
                                             "tau": "U[0.52,1.2]", "steps": "U{200..2000}"},
                "steps_per_launch": args.steps_per_launch, "budget_gib": args.budget_gib})
    print(json.dumps(rep), flush=True)
    return 0


if __name__ == "__main__":
    sys.path.insert(0, __import__("os").path.dirname(__import__("os").path.dirname(__file__)))
    raise SystemExit(main())
