"""Seeded request trace for the served form.

Independent gauge-wave evolutions arrive as a Poisson process.  Per request:
cubic edge N log-uniform in [nmin, nmax], amplitude A uniform in [amin, amax],
relaxation time tau uniform in [tmin, tmax], step count uniform in
{smin..smax}.  The wave runs along x with wavelength d = N sites.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    n: int
    amp: float
    tau: float
    steps: int


def request_trace(seed: int = 1505, rate_hz: float = 20.0, count: int = 200,
                  nmin: int = 32, nmax: int = 192,
                  amin: float = 1e-3, amax: float = 0.2,
                  tmin: float = 0.52, tmax: float = 1.2,
                  smin: int = 200, smax: int = 2000) -> list[Request]:
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    logn = rng.uniform(math.log(nmin), math.log(nmax), size=count)
    ns = np.clip(np.round(np.exp(logn)).astype(int), nmin, nmax)
    amps = rng.uniform(amin, amax, size=count)
    taus = rng.uniform(tmin, tmax, size=count)
    steps = rng.integers(smin, smax + 1, size=count)
    return [Request(i, float(arrivals[i]), int(ns[i]), float(amps[i]), float(taus[i]), int(steps[i]))
            for i in range(count)]
