"""Edge cases and host-checked failures through the C ABI on the GPU."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from paper_2201_07408_amd import _lib as L
from synth.geometry import parallel2d, cone3d
from tests.gpu_helpers import assert_close, dev, f32, host, rel

pytestmark = pytest.mark.gpu


def test_zero_rhs_gives_zero_and_no_iterations():
    desc = parallel2d(32, 20, 48)
    g = ct.Geometry(desc)
    b = torch.zeros(desc.n_rays, device="cuda")
    for fn in (ct.ct_ba_gmres, ct.ct_ab_gmres):
        r = fn(g, b, 10)
        assert r.iters_done == 0 and r.res == [0.0]
        assert torch.count_nonzero(r.x) == 0
    r = ct.ct_cgls(g, b, 10)
    assert r.iters_done == 0 and torch.count_nonzero(r.x) == 0


def test_happy_breakdown_one_pixel():
    desc = parallel2d(1, 1, 1)
    g = ct.Geometry(desc)
    r = ct.ct_ba_gmres(g, dev([2.5]), 5)
    assert r.iters_done == 1
    a = oracle.project_A(desc, np.array([1.0]))[0]
    assert abs(float(host(r.x)[0, 0, 0]) - 2.5 / a) <= 1e-6 * 2.5 / a


def test_nan_rhs_is_numeric_error():
    desc = parallel2d(16, 10, 24)
    g = ct.Geometry(desc)
    b = torch.ones(desc.n_rays, device="cuda")
    b[desc.nu // 2] = float("nan")     # a central bin of view 0: every B b sees it
    with pytest.raises(ct.CtError) as e:
        ct.ct_ba_gmres(g, b, 5)
    assert e.value.status == L.CT_ERR_NUMERIC


def test_workspace_too_small_and_bad_args():
    desc = parallel2d(16, 10, 24)
    g = ct.Geometry(desc)
    lib = L.load()
    b = torch.ones(desc.n_rays, device="cuda")
    x = torch.empty(desc.vol_shape, device="cuda")
    opts = L.SolverOpts(5, L.CT_B_UNMATCHED, L.CT_F32, 0.0)
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    st = lib.ct_ba_gmres(g.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                         ctypes.byref(opts), ctypes.c_void_p(ws.data_ptr()), 64, None, None, None)
    assert st == L.CT_ERR_ARG
    assert "workspace" in ct.ct_last_error()
    opts = L.SolverOpts(200, L.CT_B_UNMATCHED, L.CT_F32, 0.0)
    n = ctypes.c_size_t()
    assert lib.ct_solver_workspace_bytes(g.handle, L.CT_SOLVER_BA, ctypes.byref(opts),
                                         ctypes.byref(n)) == L.CT_ERR_UNSUPPORTED
    st = lib.ct_project_A(g.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                          7, 1, ctypes.c_void_p(ws.data_ptr()), 64, None)
    assert st == L.CT_ERR_ARG


def test_iteration_zero_and_max():
    desc = parallel2d(24, 30, 36)
    g = ct.Geometry(desc)
    rng = np.random.default_rng(3)
    b = f32(rng.uniform(size=desc.n_rays))
    r0 = ct.ct_ba_gmres(g, dev(b), 0)
    assert r0.iters_done == 0 and torch.count_nonzero(r0.x) == 0
    r = ct.ct_ba_gmres(g, dev(b), 56)
    ref = oracle.ba_gmres(desc, b, 56)
    assert r.iters_done == ref.iters_done
    assert rel(np.array(r.res), np.array(ref.res)) <= 1e-3


def test_views_and_detector_edges_cone():
    """Voxels that project partly off the detector (narrow detector)."""
    desc = cone3d(24, 10, 20)
    g = ct.Geometry(desc)
    y = f32(np.random.default_rng(9).uniform(size=desc.sino_shape))
    x = host(ct.ct_backproject_B(g, dev(y)))
    assert_close(x, oracle.backproject_Bun(desc, y), 1e-5, "edge B_un")
    v = f32(np.random.default_rng(10).uniform(size=desc.vol_shape))
    assert_close(host(ct.ct_project_A(g, dev(v))), oracle.project_A(desc, v), 1e-5, "edge A")
