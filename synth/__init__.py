"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package only simulates the instrument (the data model of Sec. I of the
paper: random planar array, sky of independent sources, complex-Gaussian
samples, sample covariance).  It contains none of the image-formation
arithmetic (no dirty images, bounds, operators or solvers), so that the oracle
and the GPU path can both consume its outputs without sharing any code.
"""

from .scenes import (  # noqa: F401
    CONFIGS,
    Scene,
    make_scene,
    make_request_scenes,
    make_block_scenes,
    make_offgrid_scene,
    exact_covariance,
)
