"""Seeded synthetic inputs shared by the GPU path's callers and the oracle's tests.

This package holds closed-form initial data (the gauge and linear waves and
the FLRW universe of the paper's validation section, with the FLRW fluid's
density and pressure), seeded noise and seeded request traces.  It holds
none of the lattice Boltzmann arithmetic: no equilibria, no sources, no
streaming.  Every array it returns is float64 with the field-major layout
``u[field, z, y, x]`` (x fastest) that both the oracle and the C-ABI take.

Field order (16 evolved fields per site):
    0        lapse alpha
    1..6     3-metric gamma_ij   (xx, xy, xz, yy, yz, zz)
    7..12    extrinsic curvature K_ij (same symmetric order)
    13..15   momentum variable V_k (x, y, z)
"""

from .gauge import (  # noqa: F401
    NFIELDS,
    FIELD_NAMES,
    SYM_PAIRS,
    gauge_wave_x,
    gauge_wave_diag,
    gauge_wave_dir,
    linear_wave_x,
    minkowski,
    add_lapse_noise,
    random_state,
    random_matter,
    crossing_steps_x,
    crossing_steps_diag,
)
from .flrw import flrw_exact, flrw_fields, flrw_fluid  # noqa: F401
from .trace import request_trace  # noqa: F401
