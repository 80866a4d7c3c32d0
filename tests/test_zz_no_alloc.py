"""The allocation-free forward projection (ct_project_A_noalloc) through the
C ABI against ct_project_A with a caller workspace: the same kernels, so
the same bits, over two calls in a row (the second with a smaller volume,
whose padded copies overlay what the first left in the shared scratch),
FP16 output, a batch, a 2D geometry, and the size limit (a host-side
error, no kernel launched)."""

import ctypes

import numpy as np
import pytest
import torch

import paper_2201_07408_amd as ct
from paper_2201_07408_amd import _lib as L
from synth import workloads
from synth.geometry import cone3d, parallel2d
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _noalloc(g, x, y_dtype=torch.float32, batch=1):
    lib = L.load()
    out = torch.empty((batch,) + g.sino_shape if batch > 1 else g.sino_shape, dtype=y_dtype, device="cuda")
    st = lib.ct_project_A_noalloc(g.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  L.CT_F16 if y_dtype == torch.float16 else L.CT_F32, batch,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, out


def _volume(desc, seed, batch=None):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    shape = desc.vol_shape if batch is None else (batch,) + desc.vol_shape
    return torch.rand(shape, device="cuda", generator=gen)


def test_two_calls_in_a_row_match_the_workspace_entry_point():
    big = workloads.w2_geometry()                    # 128^3, 180 views, 192^2
    small = cone3d(40, 30, 60, nz=33, nv=50)         # smaller, ragged
    gb, gs = ct.Geometry(big), ct.Geometry(small)
    xb, xs = _volume(big, 1), _volume(small, 2)
    say("no-alloc A: 128^3")
    st, yb = _noalloc(gb, xb)
    assert st == L.CT_OK, ct.ct_last_error()
    say("no-alloc A: smaller volume next")
    st, ys = _noalloc(gs, xs)
    assert st == L.CT_OK, ct.ct_last_error()
    torch.cuda.synchronize()
    assert torch.equal(yb, ct.ct_project_A(gb, xb))
    assert torch.equal(ys, ct.ct_project_A(gs, xs))
    assert float(yb.abs().max()) > 0.0 and float(ys.abs().max()) > 0.0


def test_half_output_batch_and_2d():
    desc = cone3d(24, 20, 36)
    g = ct.Geometry(desc)
    x = _volume(desc, 3, batch=3)
    say("no-alloc A: FP16 output, batch of 3")
    st, y = _noalloc(g, x, torch.float16, batch=3)
    assert st == L.CT_OK, ct.ct_last_error()
    assert torch.equal(y, ct.ct_project_A(g, x, y_dtype=torch.float16))
    d2 = parallel2d(64, 90, 96)
    g2 = ct.Geometry(d2)
    x2 = _volume(d2, 4)
    say("no-alloc A: 2D")
    st, y2 = _noalloc(g2, x2)
    assert st == L.CT_OK, ct.ct_last_error()
    assert torch.equal(y2, ct.ct_project_A(g2, x2))


def test_beyond_the_scratch_size_is_rejected_on_the_host():
    desc = cone3d(300, 4, 64)                        # padded copies of 300^3: 219 MB
    g = ct.Geometry(desc)
    lib = L.load()
    n = ctypes.c_size_t()
    assert lib.ct_op_workspace_bytes(g.handle, L.CT_OP_A, 1, ctypes.byref(n)) == L.CT_OK
    assert n.value > L.CT_NOALLOC_SCRATCH_BYTES
    x = torch.zeros(desc.vol_shape, device="cuda")
    y = torch.empty(desc.sino_shape, device="cuda")
    st = lib.ct_project_A_noalloc(g.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                  L.CT_F32, 1, None)
    assert st == L.CT_ERR_UNSUPPORTED
    assert "scratch" in ct.ct_last_error()
