"""MI355X (gfx950) lattice Boltzmann step for the Bona-Masso Einstein system.

The compute path is the HIP library ``liblbnr.so`` behind the C-ABI in
``include/lb.h``; :mod:`paper_1505_02037_amd.lb` is its ctypes binding.
"""

from .lb import (  # noqa: F401
    FP32_DEV,
    FP64,
    GEODESIC,
    HARMONIC,
    LBError,
    Lattice,
    device_bytes,
    load_library,
)
