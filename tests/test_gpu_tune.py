"""Launch settings of the cone-beam forward projector (the order in which
its ray tiles are dealt to the XCDs, and resident workgroups per CU) and
the autotuner that picks one.  A setting only reorders the workgroups, so
every setting must give bit-identical projections and solves."""

import pytest
import torch

import paper_2201_07408_amd as ct
from synth.geometry import cone3d, parallel2d
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

# XCD order with groups of 1..64 views, with and without an occupancy cap,
# and the band order with groups of 1..16 views
SETTINGS = [(1, 0), (3, 0), (10, 0), (16, 0), (64, 0), (10, 2), (-1, 0), (-2, 4), (-4, 3), (-6, 8), (-16, 1)]


def _geometry(projector):
    # ragged volume and detector: partial tiles, and view groups that do
    # not divide the 30 views
    return cone3d(40, 30, 52, nz=28, nv=44, projector=projector)


@pytest.mark.parametrize("projector", [0, 1])
def test_every_setting_gives_the_same_projection(projector):
    desc = _geometry(projector)
    g = ct.Geometry(desc)
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.rand(g.vol_shape, device="cuda", generator=gen)
    assert ct.ct_projector_get_config(g) == (10, 0)   # the size heuristic for a cached volume
    ref = ct.ct_project_A(g, x)
    ref16 = ct.ct_project_A(g, x, y_dtype=torch.float16)
    for v, w in SETTINGS:
        ct.ct_projector_config(g, v, w)
        assert ct.ct_projector_get_config(g) == (v, w)
        y = ct.ct_project_A(g, x)
        y16 = ct.ct_project_A(g, x, y_dtype=torch.float16)
        torch.cuda.synchronize()
        say("setting", (v, w), "max |y - y_default|", float((y - ref).abs().max()))
        assert torch.equal(y, ref), (v, w)
        assert torch.equal(y16, ref16), (v, w)
    ct.ct_projector_config(g, 0, 0)
    assert ct.ct_projector_get_config(g) == (10, 0)


def test_solve_under_the_band_order_matches_the_default():
    desc = _geometry(0)
    g = ct.Geometry(desc)
    gen = torch.Generator(device="cuda").manual_seed(6)
    b = ct.ct_project_A(g, torch.rand(g.vol_shape, device="cuda", generator=gen))
    r0 = ct.ct_ba_gmres(g, b, 8, B="ramp")
    ct.ct_projector_config(g, -4, 4)
    r1 = ct.ct_ba_gmres(g, b, 8, B="ramp")
    ct.ct_projector_config(g, 0, 0)
    assert torch.equal(r0.x, r1.x)
    assert r0.res == r1.res


def test_tuner_keeps_its_fastest_candidate():
    desc = _geometry(0)
    g = ct.Geometry(desc)
    gen = torch.Generator(device="cuda").manual_seed(7)
    x = torch.rand(g.vol_shape, device="cuda", generator=gen)
    ref = ct.ct_project_A(g, x)
    timed, chosen = ct.ct_tune_projector(g, reps=2)
    say("tuner", timed, "chosen", chosen)
    # a volume that fits the last-level cache: the six XCD-order candidates
    assert [(v, w) for v, w, _ in timed] == [(4, 0), (6, 0), (8, 0), (10, 0), (12, 0), (16, 0)]
    assert all(t > 0.0 for _, _, t in timed)
    assert chosen == min(timed, key=lambda e: e[2])[:2]
    assert ct.ct_projector_get_config(g) == chosen
    assert torch.equal(ct.ct_project_A(g, x), ref)


def test_allocation_free_projection_under_other_settings():
    """ct_project_A_noalloc reads the same setting: under the band order
    with an occupancy cap (dynamic LDS) and under a small XCD group it
    still gives the workspace entry point's bits."""
    import ctypes
    from paper_2201_07408_amd import _lib as L
    desc = _geometry(0)
    g = ct.Geometry(desc)
    gen = torch.Generator(device="cuda").manual_seed(8)
    x = torch.rand(g.vol_shape, device="cuda", generator=gen)
    ref = ct.ct_project_A(g, x)
    lib = L.load()
    for v, w in [(-4, 3), (6, 2), (0, 0)]:
        ct.ct_projector_config(g, v, w)
        out = torch.empty(g.sino_shape, device="cuda")
        st = lib.ct_project_A_noalloc(g.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      L.CT_F32, 1, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == L.CT_OK, lib.ct_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (v, w)


def test_settings_rejected_or_ignored_where_they_do_not_apply():
    g = ct.Geometry(_geometry(0))
    for v, w in [(0, 4), (65, 0), (-17, 0), (10, 9), (10, -1)]:
        with pytest.raises(ct.CtError):
            ct.ct_projector_config(g, v, w)
    assert ct.ct_projector_get_config(g) == (10, 0)
    g2 = ct.Geometry(parallel2d(32, 20, 48))
    with pytest.raises(ct.CtError):
        ct.ct_projector_config(g2, 10, 0)
    ct.ct_projector_config(g2, 0, 0)
    assert ct.ct_projector_get_config(g2) == (0, 0)
    assert ct.ct_tune_projector(g2) == ([], (0, 0))
