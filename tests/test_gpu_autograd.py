"""Differentiation through ct_project_A (backward = hand-written A^T).

Loss 0.5 ||A x - b||^2: the gradient is A^T (A x - b).  Checked

* against the oracle's A^T on the same FP32 residual: 1e-5 in the 2-norm
  and per voxel (relative to the largest voxel);
* against central finite differences with step h = 1e-3 at 64 seeded
  voxels (the 4 x 128^3 workload).  For a quadratic loss central
  differences are exact up to rounding, and the rounding is bounded per
  voxel: with y+- = A (x +- h e_j) evaluated by the GPU in FP32 and the
  loss difference summed in FP64 on the host,
      FD_j = sum_i (y+_i - y-_i)(y+_i + y-_i - 2 b_i) / (4 h),
  only rays touched by voxel j differ between y+ and y-, and for those the
  two FP32 results carry rounding errors of at most about 2 ulp of |y_i|
  each (the final rounding to FP32 and the FP32 partial sums; the sample
  positions and weights are the same in both).  On top of that, the
  forward's FP32 weights and the transpose's differ by up to 1e-5 of a
  weight, which can only shift g_j by 1e-5 of sum_i |A_ij r_i|.  Hence
      |FD_j - g_j| <= sum_i [3 u (|y+_i| + |y-_i|) + 1e-5 |y+_i - y-_i|] |r_i| / (2 h),
  u = 2^-24, summed over the rays where y+ and y- differ.  Every one of
  the 64 voxels must lie within this bound (not the median of them).
"""

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from tests.gpu_helpers import assert_close, dev, f32, host, say

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.mark.parametrize("n,batch", [(48, 2), (128, 4)])
def test_gradient_matches_oracle_and_fd(n, batch):
    desc = workloads.w2_geometry(n, 180 if n == 128 else 60)
    say("autograd", n, batch)
    g = ct.Geometry(desc)
    x_true = np.stack([workloads.w2_phantom(401 + i, n) for i in range(batch)])
    b = ct.ct_project_A(g, dev(x_true))
    x = dev(0.5 * x_true).requires_grad_(True)
    loss = 0.5 * ((ct.project(x, g) - b) ** 2).sum()
    loss.backward()
    grad = host(x.grad)
    r = host(ct.ct_project_A(g, x.detach()) - b)
    for i in range(batch):
        ref = oracle.backproject_AT(desc, f32(r[i]))
        assert_close(grad[i], ref, 1e-5, "autograd %d^3 item %d" % (n, i))
    # central finite differences at seeded voxels, loss differences in FP64
    rng = np.random.default_rng(405)
    h = 1e-3
    idx = rng.choice(desc.n_vox, size=64 if n == 128 else 16, replace=False)
    xb = x.detach()[0].clone()
    bh = host(b[0]).reshape(-1)
    g0 = grad[0].reshape(-1)
    worst, errs = 0.0, []
    for j in idx:
        e = torch.zeros(desc.n_vox, device="cuda")
        e[j] = h
        e = e.reshape(desc.vol_shape)
        yp = host(ct.ct_project_A(g, xb + e)).reshape(-1)
        ym = host(ct.ct_project_A(g, xb - e)).reshape(-1)
        d = yp - ym
        touched = d != 0.0
        rr = 0.5 * (yp + ym) - bh
        fd = float(np.sum(d * (yp + ym - 2.0 * bh))) / (4.0 * h)
        bound = float(np.sum((3.0 * U32 * (np.abs(yp) + np.abs(ym)) + 1e-5 * np.abs(d))[touched]
                             * np.abs(rr[touched]))) / (2.0 * h)
        err = abs(fd - g0[j])
        assert np.count_nonzero(touched) > 0
        if bound == 0.0:   # every ray through the voxel has zero residual: g_j = FD_j = 0
            assert err == 0.0 and g0[j] == 0.0, (j, fd, g0[j])
            continue
        worst = max(worst, err / bound)
        errs.append(err / max(abs(g0[j]), 1e-12))
        assert err <= bound, "voxel %d: FD %.9g, gradient %.9g, |diff| %.3e > bound %.3e" % (j, fd, g0[j], err, bound)
    say("FD: worst |FD - g| / bound %.3f; relative errors median %.2e max %.2e over %d voxels"
        % (worst, np.median(errs), np.max(errs), len(idx)))
