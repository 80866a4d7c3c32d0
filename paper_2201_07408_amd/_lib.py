"""ctypes declarations of the C ABI in include/ct.h."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libctabba.so")

CT_OK, CT_ERR_ARG, CT_ERR_ALLOC, CT_ERR_HIP, CT_ERR_NUMERIC, CT_ERR_UNSUPPORTED = range(6)
CT_PARALLEL_2D, CT_CONE_CIRCULAR_3D = 0, 1
CT_JOSEPH, CT_SIDDON = 0, 1
CT_F32, CT_F16 = 0, 1
CT_B_UNMATCHED, CT_B_RAMP, CT_B_AT = 0, 1, 2
CT_SOLVER_BA, CT_SOLVER_AB, CT_SOLVER_CGLS, CT_SOLVER_BA_MONITOR, CT_SOLVER_BA_RESTARTED = 0, 1, 2, 3, 4
CT_OP_A, CT_OP_B, CT_OP_B_RAMP, CT_OP_AT, CT_OP_FBP = 0, 1, 2, 3, 4
CT_NOALLOC_SCRATCH_BYTES = 144 << 20

# every symbol the header declares
EXPORTS = [
    "ct_geometry_create", "ct_geometry_destroy", "ct_geometry_sizes",
    "ct_op_workspace_bytes", "ct_project_A", "ct_project_A_noalloc", "ct_backproject_B",
    "ct_backproject_AT", "ct_ramp_filter", "ct_fbp", "ct_solver_workspace_bytes",
    "ct_ba_gmres", "ct_ab_gmres", "ct_cgls", "ct_last_error", "ct_version", "ct_ba_gmres_monitor",
    "ct_ba_gmres_restarted",
    "ct_profile_enable", "ct_profile_reset", "ct_profile_read",
    "ct_ba_gmres_batched_workspace_bytes", "ct_ba_gmres_batched",
    "ct_batched_config", "ct_batched_last_config",
    "ct_projector_config", "ct_projector_get_config", "ct_tune_projector",
    "ct_measure_ceilings",
]


class GeometryDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("voxel", ctypes.c_double),
        ("n_views", ctypes.c_int),
        ("angles", ctypes.POINTER(ctypes.c_double)),
        ("nu", ctypes.c_int), ("nv", ctypes.c_int),
        ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("sod", ctypes.c_double), ("sdd", ctypes.c_double),
        ("projector", ctypes.c_int),
    ]


class Ceilings(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "hbm_copy_gbs", "hbm_read_gbs", "fp32_fma_tflops", "fp32_add_tflops",
        "lds_bilinear_gsps", "l2_bilinear_gsps", "lds_gather_gbs", "l2_gather_gbs", "lds_peak_gbs")]


class SolverOpts(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("B", ctypes.c_int),
        ("sino_dtype", ctypes.c_int),
        ("breakdown_tol", ctypes.c_double),
        ("basis_dtype", ctypes.c_int),
    ]


_lib = None


def load(path: str = LIBPATH):
    """Load libctabba.so; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            "libctabba.so not found at %s: build it with "
            "`python -m paper_2201_07408_amd.build` (no CPU fallback exists)" % path)
    lib = ctypes.CDLL(path)
    vp, sz, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    szp = ctypes.POINTER(ctypes.c_size_t)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    gp = vp
    sig = {
        "ct_geometry_create": ([ctypes.POINTER(GeometryDesc), ctypes.POINTER(vp)], i),
        "ct_geometry_destroy": ([gp], None),
        "ct_geometry_sizes": ([gp, szp, szp], i),
        "ct_op_workspace_bytes": ([gp, i, i, szp], i),
        "ct_project_A": ([gp, vp, vp, i, i, vp, sz, vp], i),
        "ct_project_A_noalloc": ([gp, vp, vp, i, i, vp], i),
        "ct_backproject_B": ([gp, vp, i, vp, i, i, vp, sz, vp], i),
        "ct_backproject_AT": ([gp, vp, i, vp, i, vp, sz, vp], i),
        "ct_ramp_filter": ([gp, vp, vp, i, vp], i),
        "ct_fbp": ([gp, vp, i, vp, i, vp, sz, vp], i),
        "ct_solver_workspace_bytes": ([gp, i, ctypes.POINTER(SolverOpts), szp], i),
        "ct_ba_gmres": ([gp, vp, vp, ctypes.POINTER(SolverOpts), vp, sz, dp, ip, vp], i),
        "ct_ab_gmres": ([gp, vp, vp, ctypes.POINTER(SolverOpts), vp, sz, dp, ip, vp], i),
        "ct_cgls": ([gp, vp, vp, ctypes.POINTER(SolverOpts), vp, sz, dp, ip, vp], i),
        "ct_ba_gmres_restarted": ([gp, vp, vp, ctypes.POINTER(SolverOpts), i, vp, sz, dp, ip, vp], i),
        "ct_ba_gmres_monitor": ([gp, vp, vp, vp, ctypes.POINTER(SolverOpts), vp, sz, dp, dp, dp, ip, vp], i),
        "ct_ba_gmres_batched_workspace_bytes": ([ctypes.POINTER(vp), i, ctypes.POINTER(SolverOpts), szp], i),
        "ct_ba_gmres_batched": ([ctypes.POINTER(vp), i, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                 ctypes.POINTER(SolverOpts), vp, sz, dp, ip, vp], i),
        "ct_batched_config": ([i, i, i], i),
        "ct_batched_last_config": ([ip, ip, ip], i),
        "ct_projector_config": ([gp, i, i], i),
        "ct_projector_get_config": ([gp, ip, ip], i),
        "ct_tune_projector": ([gp, i, i, ip, ip, dp, ip, vp], i),
        "ct_measure_ceilings": ([ctypes.POINTER(Ceilings), vp], i),
        "ct_profile_enable": ([i], i),
        "ct_profile_reset": ([], i),
        "ct_profile_read": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_long), dp], i),
        "ct_last_error": ([], ctypes.c_char_p),
        "ct_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib
