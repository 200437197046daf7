"""Seeded synthetic inputs for the T2-Shuffling slice reconstruction.

This package simulates the *scanner*: phantoms with per-region proton density and
T2, smooth coil maps, variable-density Poisson-disc echo masks, an exponential
decay basis, and noisy k-space samples of the true echo images.  It holds none of
the reconstruction's arithmetic (no subspace operator, no space-time kernel, no
solver) and is shared as plain input data by the oracle tests and the GPU path.
"""

from .generate import (  # noqa: F401
    CONFIGS,
    SliceSet,
    basis,
    make_config,
    make_training_chunk,
    make_training_slices,
    training_masks,
    vd_poisson_masks,
)
