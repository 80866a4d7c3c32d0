"""Differentiation through ct_project_A (backward = hand-written A^T).

Loss 0.5 ||A x - b||^2: the gradient is A^T (A x - b).  Checked against
the oracle's A^T on the same FP32 residual and against central finite
differences, which are exact for a quadratic up to rounding; the FD bound
comes from the FP32 rounding of the projections (values ~1e2 resolved to
~1e-5, differences ~1e-3 * A e_j), i.e. ~1e-2 relative.
"""

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from tests.gpu_helpers import dev, f32, host, rel, say

pytestmark = pytest.mark.gpu


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
        assert rel(grad[i], ref) <= 1e-5
    # central finite differences at seeded voxels
    rng = np.random.default_rng(405)
    h = 1e-3
    idx = rng.choice(desc.n_vox, size=16 if n == 128 else 8, replace=False)
    xb = x.detach()[0].clone()
    bb = b[0]
    errs = []
    for j in idx:
        e = torch.zeros(desc.n_vox, device="cuda")
        e[j] = h
        e = e.reshape(desc.vol_shape)
        rp = host(ct.ct_project_A(g, xb + e) - bb)
        rm = host(ct.ct_project_A(g, xb - e) - bb)
        fd = float(((rp - rm) * (rp + rm)).sum()) / (4 * h)
        errs.append(abs(fd - grad[0].reshape(-1)[j]) / max(abs(grad[0].reshape(-1)[j]), 1e-12))
    say("FD rel errors", np.max(errs))
    assert np.median(errs) <= 1e-2
