"""The 128^3 cone-beam workload (180 views of a 192 x 192 detector) at its
full size, in the launch configuration of the solvers.

The oracle's FP64 solve takes seconds per iteration here, so it is run for
two iterations and compared vector against vector; the 50-iteration runs
are checked by properties that hold at any size: monotone residual
histories whose first entry is the norm of the right-hand side and whose
last entry equals the residual recomputed from the returned iterate."""

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from tests.gpu_helpers import dev, f32, host, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    desc = workloads.w2_geometry()
    g = ct.Geometry(desc)
    vol = workloads.w2_phantom()
    b = f32(oracle.project_A(desc, vol))          # noiseless data, FP64 projection rounded once
    return desc, g, b


def test_two_iterations_match_the_oracle(c2):
    desc, g, b = c2
    say("C2 BA-GMRES k = 2 against the oracle")
    r = ct.ct_ba_gmres(g, dev(b), 2)
    ref = oracle.ba_gmres(desc, b, 2)
    assert r.iters_done == ref.iters_done == 2
    assert rel(host(r.x), ref.x) <= 1e-4
    assert rel(np.array(r.res), np.array(ref.res)) <= 1e-4


def test_ba_gmres_50_iterations_properties(c2):
    desc, g, b = c2
    say("C2 BA-GMRES(B_un) K = 50 properties")
    bd = dev(b)
    r = ct.ct_ba_gmres(g, bd, 50)
    assert r.iters_done == 50
    res = np.array(r.res)
    assert np.all(np.diff(res) <= 1e-6 * res[0])
    assert res[-1] < 0.05 * res[0]
    Bb = ct.ct_backproject_B(g, bd.reshape(desc.sino_shape))
    assert abs(float(torch.linalg.vector_norm(Bb.double())) - res[0]) <= 1e-5 * res[0]
    rr = Bb - ct.ct_backproject_B(g, ct.ct_project_A(g, r.x))
    assert abs(float(torch.linalg.vector_norm(rr.double())) - res[-1]) <= 1e-3 * res[0]


def test_cgls_AT_50_iterations_properties(c2):
    """CGLS with the matched transpose minimises ||b - A x|| over a growing
    Krylov space, so its residual cannot increase; the recurrence's last
    residual equals the recomputed one up to the drift of the short
    recurrence in FP32 vectors."""
    desc, g, b = c2
    say("C2 CGLS(A^T) K = 50 properties")
    bd = dev(b)
    r = ct.ct_cgls(g, bd, 50, B="AT")
    res = np.array(r.res)
    assert r.iters_done == 50
    assert abs(res[0] - float(np.linalg.norm(b.astype(np.float64)))) <= 1e-6 * res[0]
    assert np.all(np.diff(res) <= 1e-5 * res[0])
    true = float(torch.linalg.vector_norm((bd - ct.ct_project_A(g, r.x).reshape(-1)).double()))
    assert abs(true - res[-1]) <= 2e-2 * res[-1] + 1e-5 * res[0]
