"""Seeded synthetic workloads for structured-FISTA image restoration.

This package only *makes inputs*: true images, point spread functions, the
blurred and noisy observation, and the random start vector of the estimate
of the Lipschitz constant.  It holds none of the restoration method's
arithmetic (no Kronecker approximation, no FISTA step).  Both the FP64 oracle and the GPU
library consume exactly the arrays produced here.
"""

from .inputs import (  # noqa: F401
    BC_REFLEXIVE,
    BC_ZERO,
    WORKLOADS,
    SEED_BATCH,
    SEED_IMAGE,
    SEED_NOISE,
    SEED_POWER,
    Problem,
    add_noise,
    blur,
    config,
    gaussian_psf,
    make_image,
    motion_psf,
    power_start,
    batch_problems,
    diff_problems,
    defocus_psf,
    paper_problems,
)
