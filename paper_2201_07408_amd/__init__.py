"""MI355X (gfx950) implementation of the ABBA method's hot path.

BA-GMRES / AB-GMRES for CT with unmatched projector pairs, plus CGLS,
behind the C ABI declared in ``include/ct.h`` (library ``libctabba.so``).
The Python layer only marshals arguments; every step runs in HIP kernels.

Importing this package does not load the library; the first call does, and
fails loudly if the library was not built.
"""

from .api import (  # noqa: F401
    Geometry,
    ct_geometry_create,
    ct_project_A,
    ct_backproject_B,
    ct_backproject_AT,
    ct_ramp_filter,
    ct_fbp,
    ct_ba_gmres,
    ct_ba_gmres_monitor,
    ct_ba_gmres_restarted,
    MonitorResult,
    ct_ab_gmres,
    ct_cgls,
    ct_ba_gmres_batched,
    ct_batched_config,
    ct_batched_last_config,
    ct_projector_config,
    ct_projector_get_config,
    ct_tune_projector,
    ct_measure_ceilings,
    ct_last_error,
    CtError,
    SolveResult,
)
from .autograd import ProjectA, project  # noqa: F401
