"""MI355X-native structured FISTA (sFISTA) for Tikhonov image restoration.

The compute path is the HIP library ``libsfista.so`` (C ABI in
``include/sfista.h``); :mod:`paper_1901_00913_amd.sfista` is its binding.
"""

from .sfista import (  # noqa: F401
    BC_REFLEXIVE,
    BC_ZERO,
    PRECISIONS,
    SfistaError,
    Solver,
    kron_approx,
    lib,
)
