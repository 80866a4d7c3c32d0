"""FP64 CPU oracle for the ABBA method (BA-GMRES / AB-GMRES / CGLS with the
Joseph projector A, its exact transpose A^T, the voxel-driven back-projector
B_un and the Ram-Lak filter F).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
baseline leg of the benchmark are the only callers.  Nothing here is shared
with, imported by, or imports the HIP library.

The operators are plain C loops in ``ct_oracle.c`` (FP64, OpenMP over
independent rays, voxels and rows); the solvers below are plain numpy and
follow the algorithm description of Sec. II of the paper:

* GMRES on S x = v with a zero initial vector: the first basis vector is the
  normalised right-hand side, each iteration applies S to the newest basis
  vector, orthonormalises it against the basis (classical Gram-Schmidt run
  twice) and solves the small least-squares problem with Givens rotations;
* BA-GMRES is GMRES on B A x = B b (Eq. 5); AB-GMRES is GMRES on A B y = b
  with x = B y (Eq. 4);
* CGLS is the textbook conjugate-gradient recurrence for min ||A x - b||
  (Eq. 2) with A^T replaced by the chosen back-projector (with B = A^T it is
  pinned against LSQR; with B = B_un it minimises nothing and its iterates
  are parity unpinned beyond the recurrence's own residual identity);
* optionally GMRES keeps its basis as FP16 values (``basis="f16"``, a storage
  option of this implementation, see ``gmres``).
"""

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libctoracle.so")
_lib = None


class _Geom(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("vox", ctypes.c_double),
        ("nviews", ctypes.c_int),
        ("angles", ctypes.POINTER(ctypes.c_double)),
        ("uniform", ctypes.c_int),
        ("nu", ctypes.c_int), ("nv", ctypes.c_int),
        ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("sod", ctypes.c_double), ("sdd", ctypes.c_double),
        ("projector", ctypes.c_int),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    gp = ctypes.POINTER(_Geom)
    i64p = ctypes.POINTER(ctypes.c_int64)
    for name, args in [
        ("orc_project_A", [gp, dp, dp]),
        ("orc_backproject_AT", [gp, dp, dp]),
        ("orc_backproject_B", [gp, dp, dp]),
        ("orc_ramp", [gp, dp, dp]),
        ("orc_project_A_rays", [gp, dp, ctypes.c_long, i64p, dp]),
        ("orc_backproject_B_voxels", [gp, dp, ctypes.c_long, i64p, dp]),
    ]:
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = None
    lib.orc_count_A_updates.argtypes = [gp]
    lib.orc_count_A_updates.restype = ctypes.c_int64
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def uniform_angles(kind: int, n_views: int) -> np.ndarray:
    """t_p = pi p / P (2D parallel, half turn) or 2 pi p / P (3D cone, full
    turn), each evaluated as (c * p) / P in FP64."""
    span = math.pi if kind == 0 else 2.0 * math.pi
    return np.array([(span * p) / n_views for p in range(n_views)], dtype=np.float64)


class Geometry:
    """Holds the ctypes struct and keeps the angle array alive."""

    def __init__(self, desc):
        self.desc = desc
        if desc.angles is None:
            self.angles = uniform_angles(desc.kind, desc.n_views)
            uniform = 1
        else:
            self.angles = np.ascontiguousarray(desc.angles, dtype=np.float64)
            assert self.angles.size == desc.n_views
            uniform = 0
        self.c = _Geom(desc.kind, desc.nx, desc.ny, desc.nz, desc.voxel,
                       desc.n_views,
                       self.angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       uniform, desc.nu, desc.nv, desc.du, desc.dv,
                       desc.sod, desc.sdd, int(getattr(desc, "projector", 0)))
        self.n = desc.nx * desc.ny * desc.nz
        self.m = desc.n_views * desc.nv * desc.nu
        self.vol_shape = (desc.nz, desc.ny, desc.nx)
        self.sino_shape = (desc.n_views, desc.nv, desc.nu)


def _geom(g) -> Geometry:
    return g if isinstance(g, Geometry) else Geometry(g)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ------------------------------------------------------------- operators
def project_A(g, x) -> np.ndarray:
    """Joseph forward projection y = A x; x has g.n entries (volume order)."""
    g = _geom(g)
    x = _f64(x).reshape(-1)
    assert x.size == g.n
    y = np.empty(g.m, dtype=np.float64)
    _load().orc_project_A(ctypes.byref(g.c), _dptr(x), _dptr(y))
    return y


def project_A_rays(g, x, ray_ids) -> np.ndarray:
    g = _geom(g)
    x = _f64(x).reshape(-1)
    ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
    out = np.empty(ids.size, dtype=np.float64)
    _load().orc_project_A_rays(ctypes.byref(g.c), _dptr(x), ids.size,
                               ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               _dptr(out))
    return out


def backproject_AT(g, y) -> np.ndarray:
    g = _geom(g)
    y = _f64(y).reshape(-1)
    assert y.size == g.m
    x = np.empty(g.n, dtype=np.float64)
    _load().orc_backproject_AT(ctypes.byref(g.c), _dptr(y), _dptr(x))
    return x


def backproject_Bun(g, y) -> np.ndarray:
    g = _geom(g)
    y = _f64(y).reshape(-1)
    assert y.size == g.m
    x = np.empty(g.n, dtype=np.float64)
    _load().orc_backproject_B(ctypes.byref(g.c), _dptr(y), _dptr(x))
    return x


def backproject_Bun_voxels(g, y, vox_ids) -> np.ndarray:
    g = _geom(g)
    y = _f64(y).reshape(-1)
    ids = np.ascontiguousarray(vox_ids, dtype=np.int64)
    out = np.empty(ids.size, dtype=np.float64)
    _load().orc_backproject_B_voxels(ctypes.byref(g.c), _dptr(y), ids.size,
                                     ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     _dptr(out))
    return out


def ramp(g, y) -> np.ndarray:
    g = _geom(g)
    y = _f64(y).reshape(-1)
    assert y.size == g.m
    out = np.empty(g.m, dtype=np.float64)
    _load().orc_ramp(ctypes.byref(g.c), _dptr(y), _dptr(out))
    return out


def fbp(g, y) -> np.ndarray:
    """One-shot filtered back-projection with the paper's B_un and F (the
    reference reconstruction it compares against, Sec. III), scaled to
    approximate the inverse Radon / cone-beam transform:
      2D parallel beam:  x = (pi / P) (du / vox^2) B_un F y
         (the ramp-filtered projection interpolated at x . n and summed over
         P views spread over pi; B_un carries the weight vox^2 / du);
      3D circular cone beam (Feldkamp-Davis-Kress):
         x = (pi / P) (SOD / SDD) (du dv / vox^3) B_un F (w . y),
         w = SDD / sqrt(SDD^2 + u^2 + v^2)  (cosine pre-weighting),
         where B_un's weight vox^3 M^2 / (du dv) carries the distance factor
         (SDD / U)^2 = (SDD / SOD)^2 (SOD / U)^2 and filtering in detector
         pitch instead of isocentre pitch contributes SDD / SOD; the full
         turn of P views counts every ray twice (the 1/2 of the formula)."""
    g = _geom(g)
    d = g.desc
    y = _f64(y).reshape(d.n_views, d.nv, d.nu)
    if d.kind == 0:
        scale = (math.pi / d.n_views) * d.du / (d.voxel ** 2)
        return scale * backproject_Bun(g, ramp(g, y))
    u = (np.arange(d.nu) - 0.5 * (d.nu - 1)) * d.du
    v = (np.arange(d.nv) - 0.5 * (d.nv - 1)) * d.dv
    w = d.sdd / np.sqrt(d.sdd ** 2 + u[None, :] ** 2 + v[:, None] ** 2)
    scale = (math.pi / d.n_views) * (d.sod / d.sdd) * d.du * d.dv / (d.voxel ** 3)
    return scale * backproject_Bun(g, ramp(g, y * w[None, :, :]))


def count_A_updates(g) -> int:
    g = _geom(g)
    return int(_load().orc_count_A_updates(ctypes.byref(g.c)))


def count_B_updates(g) -> int:
    g = _geom(g)
    return int(g.n) * int(g.desc.n_views)


def back_projector(g, which: str) -> Callable[[np.ndarray], np.ndarray]:
    """'un' -> B_un, 'ramp' -> B_un F (B_FBP), 'AT' -> A^T."""
    g = _geom(g)
    if which == "un":
        return lambda y: backproject_Bun(g, y)
    if which == "ramp":
        return lambda y: backproject_Bun(g, ramp(g, y))
    if which == "AT":
        return lambda y: backproject_AT(g, y)
    raise ValueError(which)


# --------------------------------------------------------------- solvers
EPS64 = np.finfo(np.float64).eps / 2.0   # unit roundoff 2^-53


@dataclass
class GmresResult:
    x: np.ndarray                 # solution estimate (image space)
    res: List[float]              # |g_{k+1}| per step, res[0] = ||r0||
    iters_done: int
    W: Optional[np.ndarray] = None  # orthonormal basis, rows
    H: Optional[np.ndarray] = None  # upper-triangular R after rotations
    coeff: Optional[np.ndarray] = None  # y with x = W^T y (BA) / x = B W^T y (AB)


def _round16(v: np.ndarray) -> np.ndarray:
    """Values of v as stored in FP16: rounded to FP32 first (the precision
    the stored vector is computed in), then to the nearest FP16 (ties to
    even), returned as FP64."""
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def _pow2_below(norm: float, n: int) -> float:
    """The power of two t with t * norm in (sqrt(n)/2, sqrt(n)]."""
    return float(2.0 ** math.floor(math.log2(math.sqrt(n) / norm)))


def gmres(apply_S: Callable[[np.ndarray], np.ndarray], r0: np.ndarray, iters: int,
          tau: float = 64 * EPS64, keep_basis: bool = False, basis: str = "f64"):
    """GMRES with x0 = 0 on S x = r0.  Returns (coeff, W, res, iters_done, R).

    Breakdown: the step stops after column k when the new vector's norm
    after orthogonalisation is at most tau times its norm before.

    basis = "f16": the basis is kept as FP16 values (a storage choice of this
    implementation, not of the paper).  The first vector is stored as
    FP16(t0 r0) with t0 the power of two that puts t0 ||r0|| in
    (sqrt(n)/2, sqrt(n)]; each later vector as FP16(t z2), z2 the vector
    after both Gram-Schmidt passes and t chosen from the norm of the vector
    after the first pass.  The basis vector used from then on is the stored
    values divided by t times the unrounded norm, so H and the residual
    recurrence are those of the unrounded vectors, and the rounding is the
    only change."""
    r0 = np.asarray(r0, dtype=np.float64)
    beta = float(np.linalg.norm(r0))
    res = [beta]
    if beta == 0.0 or iters <= 0:
        return np.zeros(0), np.zeros((0, r0.size)), res, 0, np.zeros((0, 0))
    if basis not in ("f64", "f16"):
        raise ValueError("basis must be 'f64' or 'f16'")
    f16 = basis == "f16"
    n = r0.size
    W = np.zeros((iters + 1, r0.size), dtype=np.float64)
    if f16:
        t0 = _pow2_below(beta, n)
        W[0] = _round16(t0 * r0) / (t0 * beta)
    else:
        W[0] = r0 / beta
    H = np.zeros((iters + 1, iters), dtype=np.float64)
    cs = np.zeros(iters)
    sn = np.zeros(iters)
    gv = np.zeros(iters + 1)
    gv[0] = beta
    done = 0
    for k in range(iters):
        z = apply_S(W[k])
        znorm0 = float(np.linalg.norm(z))
        Wk = W[: k + 1]
        # classical Gram-Schmidt, twice
        h1 = Wk @ z
        z = z - Wk.T @ h1
        if f16:
            z1n = float(np.linalg.norm(z))
            t = _pow2_below(z1n, n) if z1n > 0.0 else 1.0
        h2 = Wk @ z
        z = z - Wk.T @ h2
        hnext = float(np.linalg.norm(z))
        H[: k + 1, k] = h1 + h2
        H[k + 1, k] = hnext
        # previous rotations applied to the new column
        for i in range(k):
            a, bb = H[i, k], H[i + 1, k]
            H[i, k] = cs[i] * a + sn[i] * bb
            H[i + 1, k] = -sn[i] * a + cs[i] * bb
        rho = math.hypot(H[k, k], H[k + 1, k])
        cs[k] = H[k, k] / rho
        sn[k] = H[k + 1, k] / rho
        H[k, k] = rho
        H[k + 1, k] = 0.0
        gv[k + 1] = -sn[k] * gv[k]
        gv[k] = cs[k] * gv[k]
        res.append(abs(gv[k + 1]))
        done = k + 1
        if hnext <= tau * znorm0:
            break
        W[k + 1] = _round16(t * z) / (t * hnext) if f16 else z / hnext
    R = H[:done, :done]
    coeff = np.zeros(done)
    for i in range(done - 1, -1, -1):   # back substitution
        coeff[i] = (gv[i] - R[i, i + 1: done] @ coeff[i + 1: done]) / R[i, i]
    return coeff, W[:done], res, done, R


def ba_gmres(g, b, iters: int, B: str = "un", tau: float = 64 * EPS64,
             keep_basis: bool = False, basis: str = "f64") -> GmresResult:
    """BA-GMRES (Eq. 5): GMRES on B A x = B b; x_k = W_k y_k."""
    g = _geom(g)
    Bop = back_projector(g, B)
    r0 = Bop(_f64(b).reshape(-1))
    coeff, W, res, k, R = gmres(lambda v: Bop(project_A(g, v)), r0, iters, tau, basis=basis)
    x = W.T @ coeff if k > 0 else np.zeros(g.n)
    return GmresResult(x, res, k, W if keep_basis else None, R, coeff)


def ab_gmres(g, b, iters: int, B: str = "un", tau: float = 64 * EPS64,
             keep_basis: bool = False) -> GmresResult:
    """AB-GMRES (Eq. 4): GMRES on A B y = b; x_k = B (W_k c_k)."""
    g = _geom(g)
    Bop = back_projector(g, B)
    r0 = _f64(b).reshape(-1)
    coeff, W, res, k, R = gmres(lambda v: project_A(g, Bop(v)), r0, iters, tau)
    x = Bop(W.T @ coeff) if k > 0 else np.zeros(g.n)
    return GmresResult(x, res, k, W if keep_basis else None, R, coeff)


@dataclass
class CglsResult:
    x: np.ndarray
    res: List[float]        # ||r_k|| = ||b - A x_k|| from the recurrence
    iters_done: int


def cgls(g, b, iters: int, B: str = "AT") -> CglsResult:
    """CGLS for Eq. 2 with the back-projector B in the place of A^T.
    B = "AT": pinned (equals LSQR); B = "un": parity unpinned beyond the
    recursive residual tracking ||b - A x_k||."""
    g = _geom(g)
    Bop = back_projector(g, B)
    b = _f64(b).reshape(-1)
    x = np.zeros(g.n)
    r = b.copy()
    s = Bop(r)
    p = s.copy()
    gamma = float(s @ s)
    res = [float(np.linalg.norm(r))]
    done = 0
    for _ in range(iters):
        if gamma == 0.0:
            break
        q = project_A(g, p)
        qq = float(q @ q)
        if qq == 0.0:
            break
        alpha = gamma / qq
        x = x + alpha * p
        r = r - alpha * q
        s = Bop(r)
        gamma_new = float(s @ s)
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        res.append(float(np.linalg.norm(r)))
        done += 1
    return CglsResult(x, res, done)


def ba_gmres_restarted(g, b, m: int, cycles: int, B: str = "un", basis: str = "f64"):
    """Restarted BA-GMRES(m): each cycle runs m steps of BA-GMRES on the
    data residual of the current iterate and adds the correction
    (x <- x + d, d from K_m(BA, B(b - A x))).  Returns (x, list of the
    cycles' residual histories)."""
    g = _geom(g)
    b = _f64(b).reshape(-1)
    x = np.zeros(g.n)
    hist = []
    for _ in range(cycles):
        r = b - np.asarray(project_A(g, x.reshape(g.vol_shape))).reshape(-1)
        res = ba_gmres(g, r, m, B=B, basis=basis)
        x = x + np.asarray(res.x).reshape(-1)
        hist.append(list(res.res))
    return x, hist
