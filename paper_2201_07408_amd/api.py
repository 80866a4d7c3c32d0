"""Python binding of the C ABI (argument marshalling only).

Tensors are torch device tensors; the work is enqueued on torch's current
stream of the tensors' device.  Function names follow include/ct.h.
"""

import ctypes
from dataclasses import dataclass
from typing import List, Optional

import torch

from . import _lib as L


class CtError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = ct_last_error()
        super().__init__("%s failed with status %d: %s" % (where, status, msg))
        self.status = status


def ct_last_error() -> str:
    v = L.load().ct_last_error()
    return v.decode() if v else ""


def _check(status: int, where: str) -> None:
    if status != L.CT_OK:
        raise CtError(status, where)


def _stream(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _need_device(t: torch.Tensor, name: str, dtype=None) -> None:
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor (no CPU path exists)" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))


_DT = {torch.float32: L.CT_F32, torch.float16: L.CT_F16}
_B = {"un": L.CT_B_UNMATCHED, "ramp": L.CT_B_RAMP, "AT": L.CT_B_AT}


class Geometry:
    """Owns a ct_geometry handle.  `desc` is any object with the fields of
    ct_geometry_desc (kind, nx, ny, nz, voxel, n_views, nu, nv, du, dv, sod,
    sdd, angles)."""

    def __init__(self, desc, device=None):
        lib = L.load()
        self.desc = desc
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        angles = getattr(desc, "angles", None)
        self._angles = None
        ap = None
        if angles is not None:
            self._angles = (ctypes.c_double * len(angles))(*[float(a) for a in angles])
            ap = ctypes.cast(self._angles, ctypes.POINTER(ctypes.c_double))
        d = L.GeometryDesc(int(desc.kind), int(desc.nx), int(desc.ny), int(desc.nz),
                           float(desc.voxel), int(desc.n_views), ap, int(desc.nu),
                           int(desc.nv), float(desc.du), float(desc.dv),
                           float(getattr(desc, "sod", 0.0)), float(getattr(desc, "sdd", 0.0)),
                           int(getattr(desc, "projector", 0)))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.ct_geometry_create(ctypes.byref(d), ctypes.byref(h)), "ct_geometry_create")
        self.handle = h
        self._lib = lib
        nv, nr = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib.ct_geometry_sizes(h, ctypes.byref(nv), ctypes.byref(nr)), "ct_geometry_sizes")
        self.n_vox, self.n_rays = nv.value, nr.value
        self.vol_shape = (int(desc.nz), int(desc.ny), int(desc.nx))
        self.sino_shape = (int(desc.n_views), int(desc.nv), int(desc.nu))
        self._ws = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        lib = getattr(self, "_lib", None)
        if h is None or not h.value or lib is None:
            return
        try:
            torch.cuda.synchronize(self.device)
            lib.ct_geometry_destroy(h)
        except Exception:
            pass   # interpreter shutdown: the process releases the memory
        self.handle = None

    # workspace cache: one buffer per purpose, grown on demand
    def workspace(self, key: str, nbytes: int) -> torch.Tensor:
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def op_workspace(self, op: int, batch: int = 1) -> torch.Tensor:
        n = ctypes.c_size_t()
        _check(L.load().ct_op_workspace_bytes(self.handle, op, batch, ctypes.byref(n)),
               "ct_op_workspace_bytes")
        return self.workspace("op%d" % op, n.value)


def ct_geometry_create(desc, device=None) -> Geometry:
    return Geometry(desc, device)


def _batch_of(t: torch.Tensor, item_numel: int, name: str) -> int:
    if t.numel() % item_numel != 0 or t.numel() == 0 and item_numel == 0:
        raise ValueError("%s has %d elements, not a multiple of %d" % (name, t.numel(), item_numel))
    return t.numel() // item_numel


def ct_project_A(g: Geometry, x: torch.Tensor, y_dtype=torch.float32,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = A x; x [..., nz, ny, nx] float32 -> y [..., P, nv, nu]."""
    _need_device(x, "x", torch.float32)
    batch = _batch_of(x, g.n_vox, "x")
    lead = x.shape[:-3] if x.dim() >= 3 else ()
    if out is None:
        out = torch.empty(tuple(lead) + g.sino_shape, dtype=y_dtype, device=x.device)
    _need_device(out, "out", y_dtype)
    ws = g.op_workspace(L.CT_OP_A, batch)
    _check(L.load().ct_project_A(g.handle, _ptr(x), _ptr(out), _DT[y_dtype], batch, _ptr(ws),
                                 ws.numel(), _stream(x)), "ct_project_A")
    return out


def ct_backproject_B(g: Geometry, y: torch.Tensor, ramp: bool = False,
                     out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = B_un y (ramp=False) or B_un F y (ramp=True)."""
    _need_device(y, "y")
    batch = _batch_of(y, g.n_rays, "y")
    lead = y.shape[:-3] if y.dim() >= 3 else ()
    if out is None:
        out = torch.empty(tuple(lead) + g.vol_shape, dtype=torch.float32, device=y.device)
    _need_device(out, "out", torch.float32)
    ws = g.op_workspace(L.CT_OP_B_RAMP if ramp else L.CT_OP_B, batch)
    _check(L.load().ct_backproject_B(g.handle, _ptr(y), _DT[y.dtype], _ptr(out), int(bool(ramp)),
                                     batch, _ptr(ws), ws.numel(), _stream(y)), "ct_backproject_B")
    return out


def ct_backproject_AT(g: Geometry, y: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = A^T y (exact transpose of ct_project_A)."""
    _need_device(y, "y")
    batch = _batch_of(y, g.n_rays, "y")
    lead = y.shape[:-3] if y.dim() >= 3 else ()
    if out is None:
        out = torch.empty(tuple(lead) + g.vol_shape, dtype=torch.float32, device=y.device)
    _need_device(out, "out", torch.float32)
    ws = g.op_workspace(L.CT_OP_AT, batch)
    _check(L.load().ct_backproject_AT(g.handle, _ptr(y), _DT[y.dtype], _ptr(out), batch, _ptr(ws),
                                      ws.numel(), _stream(y)), "ct_backproject_AT")
    return out


def ct_fbp(g: Geometry, y: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One-shot FBP (2D) / FDK (cone) reconstruction from B_un and F."""
    _need_device(y, "y")
    batch = _batch_of(y, g.n_rays, "y")
    lead = y.shape[:-3] if y.dim() >= 3 else ()
    if out is None:
        out = torch.empty(tuple(lead) + g.vol_shape, dtype=torch.float32, device=y.device)
    _need_device(out, "out", torch.float32)
    ws = g.op_workspace(L.CT_OP_FBP, batch)
    _check(L.load().ct_fbp(g.handle, _ptr(y), _DT[y.dtype], _ptr(out), batch, _ptr(ws), ws.numel(),
                           _stream(y)), "ct_fbp")
    return out


def ct_ramp_filter(g: Geometry, q: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    _need_device(q, "q", torch.float32)
    batch = _batch_of(q, g.n_rays, "q")
    if out is None:
        out = torch.empty_like(q)
    _check(L.load().ct_ramp_filter(g.handle, _ptr(q), _ptr(out), batch, _stream(q)), "ct_ramp_filter")
    return out


@dataclass
class SolveResult:
    x: torch.Tensor
    res: List[float]
    iters_done: int


def _solve(fn_name: str, solver: int, g: Geometry, b: torch.Tensor, iters: int, B: str,
           sino_dtype, breakdown_tol: float, out: Optional[torch.Tensor],
           basis_dtype=torch.float32) -> SolveResult:
    _need_device(b, "b", torch.float32)
    if b.numel() != g.n_rays:
        raise ValueError("b must have %d elements" % g.n_rays)
    lib = L.load()
    opts = L.SolverOpts(int(iters), _B[B], _DT[sino_dtype], float(breakdown_tol), _DT[basis_dtype])
    n = ctypes.c_size_t()
    _check(lib.ct_solver_workspace_bytes(g.handle, solver, ctypes.byref(opts), ctypes.byref(n)),
           "ct_solver_workspace_bytes")
    ws = g.workspace("solver", n.value)
    if out is None:
        out = torch.empty(g.vol_shape, dtype=torch.float32, device=b.device)
    _need_device(out, "out", torch.float32)
    res = (ctypes.c_double * (int(iters) + 1))()
    done = ctypes.c_int(0)
    st = getattr(lib, fn_name)(g.handle, _ptr(b), _ptr(out), ctypes.byref(opts), _ptr(ws), ws.numel(),
                               res, ctypes.byref(done), _stream(b))
    _check(st, fn_name)
    return SolveResult(out, list(res)[: done.value + 1], done.value)


def ct_ba_gmres(g: Geometry, b: torch.Tensor, iters: int, B: str = "un", sino_dtype=torch.float32,
                breakdown_tol: float = 0.0, out: Optional[torch.Tensor] = None,
                basis_dtype=torch.float32) -> SolveResult:
    """BA-GMRES (Eq. 5): GMRES on B A x = B b, x0 = 0.  basis_dtype =
    torch.float16 stores the Krylov basis in FP16 (power-of-two scaled)."""
    return _solve("ct_ba_gmres", L.CT_SOLVER_BA, g, b, iters, B, sino_dtype, breakdown_tol, out, basis_dtype)


@dataclass
class RestartResult:
    x: torch.Tensor
    res: List[List[float]]     # per cycle, as ct_ba_gmres's history
    iters_done: int


def ct_ba_gmres_restarted(g: Geometry, b: torch.Tensor, m: int, cycles: int, B: str = "un",
                          breakdown_tol: float = 0.0, out: Optional[torch.Tensor] = None,
                          basis_dtype=torch.float32) -> RestartResult:
    """Restarted BA-GMRES(m): `cycles` cycles of m steps on the data residual."""
    _need_device(b, "b", torch.float32)
    if b.numel() != g.n_rays:
        raise ValueError("b must have %d elements" % g.n_rays)
    lib = L.load()
    opts = L.SolverOpts(int(m), _B[B], L.CT_F32, float(breakdown_tol), _DT[basis_dtype])
    n = ctypes.c_size_t()
    _check(lib.ct_solver_workspace_bytes(g.handle, L.CT_SOLVER_BA_RESTARTED, ctypes.byref(opts), ctypes.byref(n)),
           "ct_solver_workspace_bytes")
    ws = g.workspace("restarted", n.value)
    if out is None:
        out = torch.empty(g.vol_shape, dtype=torch.float32, device=b.device)
    _need_device(out, "out", torch.float32)
    K1 = int(m) + 1
    res = (ctypes.c_double * (K1 * int(cycles)))()
    done = ctypes.c_int(0)
    _check(lib.ct_ba_gmres_restarted(g.handle, _ptr(b), _ptr(out), ctypes.byref(opts), int(cycles), _ptr(ws),
                                     ws.numel(), res, ctypes.byref(done), _stream(b)), "ct_ba_gmres_restarted")
    hist = [[v for v in res[c * K1:(c + 1) * K1] if v == v] for c in range(int(cycles))]
    return RestartResult(out, hist, done.value)


@dataclass
class MonitorResult:
    x: torch.Tensor
    res: List[float]
    data_res: List[float]      # ||b - A x_k||, k = 0..iters_done
    img_rmse: List[float]      # RMSE(x_k - x_ref) (NaN without x_ref)
    iters_done: int


def ct_ba_gmres_monitor(g: Geometry, b: torch.Tensor, iters: int, B: str = "un",
                        x_ref: Optional[torch.Tensor] = None, breakdown_tol: float = 0.0,
                        out: Optional[torch.Tensor] = None) -> MonitorResult:
    """BA-GMRES with the per-iteration data residual and image error."""
    _need_device(b, "b", torch.float32)
    if b.numel() != g.n_rays:
        raise ValueError("b must have %d elements" % g.n_rays)
    if x_ref is not None:
        _need_device(x_ref, "x_ref", torch.float32)
        if x_ref.numel() != g.n_vox:
            raise ValueError("x_ref must have %d elements" % g.n_vox)
    lib = L.load()
    opts = L.SolverOpts(int(iters), _B[B], L.CT_F32, float(breakdown_tol))
    n = ctypes.c_size_t()
    _check(lib.ct_solver_workspace_bytes(g.handle, L.CT_SOLVER_BA_MONITOR, ctypes.byref(opts), ctypes.byref(n)),
           "ct_solver_workspace_bytes")
    ws = g.workspace("monitor", n.value)
    if out is None:
        out = torch.empty(g.vol_shape, dtype=torch.float32, device=b.device)
    _need_device(out, "out", torch.float32)
    K1 = int(iters) + 1
    res, dres, img = (ctypes.c_double * K1)(), (ctypes.c_double * K1)(), (ctypes.c_double * K1)()
    done = ctypes.c_int(0)
    st = lib.ct_ba_gmres_monitor(g.handle, _ptr(b), _ptr(out), None if x_ref is None else _ptr(x_ref),
                                 ctypes.byref(opts), _ptr(ws), ws.numel(), res, dres, img,
                                 ctypes.byref(done), _stream(b))
    _check(st, "ct_ba_gmres_monitor")
    k = done.value + 1
    return MonitorResult(out, list(res)[:k], list(dres)[:k], list(img)[:k], done.value)


def ct_ab_gmres(g: Geometry, b: torch.Tensor, iters: int, B: str = "un", breakdown_tol: float = 0.0,
                out: Optional[torch.Tensor] = None) -> SolveResult:
    """AB-GMRES (Eq. 4): GMRES on A B y = b, x = B y."""
    return _solve("ct_ab_gmres", L.CT_SOLVER_AB, g, b, iters, B, torch.float32, breakdown_tol, out)


def ct_cgls(g: Geometry, b: torch.Tensor, iters: int, B: str = "AT",
            out: Optional[torch.Tensor] = None) -> SolveResult:
    """CGLS (Eq. 2) with A^T replaced by B."""
    return _solve("ct_cgls", L.CT_SOLVER_CGLS, g, b, iters, B, torch.float32, 0.0, out)


_BATCH_WS = {}


def ct_ba_gmres_batched(geoms: List[Geometry], bs: List[torch.Tensor], iters: int, B: str = "un",
                        breakdown_tol: float = 0.0,
                        outs: Optional[List[torch.Tensor]] = None) -> List[SolveResult]:
    """BA-GMRES (Eq. 5) on many independent 2D problems in one batched solve."""
    count = len(geoms)
    if len(bs) != count:
        raise ValueError("one data array per geometry")
    if count == 0:
        return []
    for i, (g, b) in enumerate(zip(geoms, bs)):
        _need_device(b, "b[%d]" % i, torch.float32)
        if b.numel() != g.n_rays:
            raise ValueError("b[%d] must have %d elements" % (i, g.n_rays))
    if outs is None:
        outs = [torch.empty(g.vol_shape, dtype=torch.float32, device=b.device) for g, b in zip(geoms, bs)]
    for i, (g, x) in enumerate(zip(geoms, outs)):
        _need_device(x, "x[%d]" % i, torch.float32)
        if x.numel() != g.n_vox:
            raise ValueError("x[%d] must have %d elements" % (i, g.n_vox))
    lib = L.load()
    opts = L.SolverOpts(int(iters), _B[B], L.CT_F32, float(breakdown_tol))
    garr = (ctypes.c_void_p * count)(*[g.handle.value for g in geoms])
    barr = (ctypes.c_void_p * count)(*[b.data_ptr() for b in bs])
    xarr = (ctypes.c_void_p * count)(*[x.data_ptr() for x in outs])
    n = ctypes.c_size_t()
    _check(lib.ct_ba_gmres_batched_workspace_bytes(garr, count, ctypes.byref(opts), ctypes.byref(n)),
           "ct_ba_gmres_batched_workspace_bytes")
    dev = bs[0].device
    ws = _BATCH_WS.get(dev)
    if ws is None or ws.numel() < n.value:
        _BATCH_WS.pop(dev, None)
        ws = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=dev)
        _BATCH_WS[dev] = ws
    K1 = int(iters) + 1
    res = (ctypes.c_double * (count * K1))()
    done = (ctypes.c_int * count)()
    _check(lib.ct_ba_gmres_batched(garr, count, barr, xarr, ctypes.byref(opts), _ptr(ws), ws.numel(),
                                   res, done, _stream(bs[0])), "ct_ba_gmres_batched")
    return [SolveResult(outs[i], list(res[i * K1: i * K1 + done[i] + 1]), int(done[i])) for i in range(count)]


def ct_batched_config(use_graph: bool = True, a_variant: int = -1, b_variant: int = -1) -> None:
    _check(L.load().ct_batched_config(int(bool(use_graph)), int(a_variant), int(b_variant)), "ct_batched_config")


def ct_projector_config(g: Geometry, vgrp: int = 0, wg_per_cu: int = 0) -> None:
    """Launch setting of the cone-beam forward projector of `g` (0, 0: the
    size heuristic); every setting gives bit-identical results."""
    _check(L.load().ct_projector_config(g.handle, int(vgrp), int(wg_per_cu)), "ct_projector_config")


def ct_projector_get_config(g: Geometry):
    """(vgrp, wg_per_cu) in use by the forward projector of `g`."""
    v, w = ctypes.c_int(), ctypes.c_int()
    _check(L.load().ct_projector_get_config(g.handle, ctypes.byref(v), ctypes.byref(w)), "ct_projector_get_config")
    return v.value, w.value


def ct_tune_projector(g: Geometry, reps: int = 3, cap: int = 32):
    """Time the forward projector's launch settings on `g` (on the current
    stream of g's device) and keep the fastest; returns the list of
    (vgrp, wg_per_cu, ms per launch) timed and the setting chosen."""
    v = (ctypes.c_int * cap)()
    w = (ctypes.c_int * cap)()
    t = (ctypes.c_double * cap)()
    n = ctypes.c_int()
    with torch.cuda.device(g.device):
        st = ctypes.c_void_p(torch.cuda.current_stream(g.device).cuda_stream)
        _check(L.load().ct_tune_projector(g.handle, int(reps), int(cap), v, w, t, ctypes.byref(n), st),
               "ct_tune_projector")
    timed = [(v[i], w[i], t[i]) for i in range(min(n.value, cap))]
    return timed, ct_projector_get_config(g)


def ct_measure_ceilings(device=None) -> dict:
    """Measured ceilings of the device (HBM copy and read rates, FP32 FMA
    and add rates, bilinear samples per second from LDS and from L2), on
    the device's current stream."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    c = L.Ceilings()
    with torch.cuda.device(dev):
        st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        _check(L.load().ct_measure_ceilings(ctypes.byref(c), st), "ct_measure_ceilings")
    return {name: getattr(c, name) for name, _ in L.Ceilings._fields_}


def ct_batched_last_config():
    g, a, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(L.load().ct_batched_last_config(ctypes.byref(g), ctypes.byref(a), ctypes.byref(b)),
           "ct_batched_last_config")
    return bool(g.value), a.value, b.value
