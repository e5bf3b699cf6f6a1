"""Seeded synthetic inputs for the FFT-convolution CG solver.

This package holds only input recipes: the kernel spectrum of the synthetic
long-range kernel, the per-instance diagonal ``d``, right-hand side ``b``,
thresholds ``t`` and the serving arrival schedule.  It contains none of the
solver's arithmetic (no convolution, no FFT, no CG), so both the CPU oracle
and the GPU path may draw their inputs from it.
"""

from .configs import (  # noqa: F401
    spectrum,
    periodic_instance,
    padded_instance,
    c1_instance,
    c2_instance,
    c3_instance,
    c4_schedule,
    c4_request,
    c5_sequence,
    fracture_instance,
    CONFIGS,
)
