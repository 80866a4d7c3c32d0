"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds no part of the reconstruction method: no projector, no
back-projector, no filter and no solver.  It only describes geometries
(sizes and angles) and draws phantoms and noise from fixed seeds, so that the
HIP path and the CPU oracle can be fed the very same arrays.
"""

from .geometry import GeometryDesc, PARALLEL_2D, CONE_3D  # noqa: F401
from .phantoms import (  # noqa: F401
    random_ellipses,
    random_ellipsoids,
    rasterize_ellipses,
    rasterize_ellipsoids,
    smooth_texture,
    gaussian_noise,
    poisson_log_counts,
)
from . import workloads  # noqa: F401
