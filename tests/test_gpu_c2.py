"""The 128^3 cone-beam workload (180 views of a 192 x 192 detector) at its
full size, in the launch configuration of the solvers, against the FP64
oracle at the iteration counts of the workload (Sec. II, Eq. 5; Sec. I,
Eq. 2).

Data: noiseless b = A x_true with the oracle's projector, rounded once to
FP32 (both sides read the same FP32 values).

* BA-GMRES(B_un), K = 50: the iterate and every entry of the residual
  history against the oracle's, at 1e-4.  Noiseless data leave the exact
  iterate insensitive to FP32-sized perturbations of the operators at this
  K (the sensitivity that forces the FP32 envelope on the noisy 2D problem
  does not arise here).
* CGLS(A^T), K = 50: a short recurrence, whose iterates in FP32 can drift
  from the FP64 ones as the recurrence loses conjugacy (on the noisy 2D
  problem by 1e-2 at k = 10).  On these noiseless data the oracle's own
  recurrence with every vector rounded to FP32 at each step, and its
  operator outputs perturbed at FP32 accumulation size, moves x_50 by
  1.8e-6 and the residuals by at most 1.3e-7 (tests/golden/
  cgls_fp32_spread.json, written by tests/golden/make_cgls_spread.py from
  the oracle alone), so the iterate and every residual entry are held to
  1e-4, or three times that spread if it were larger.
* Both: properties at any size (monotone histories, first entry the norm of
  the right-hand side, last entry the recomputed residual of the returned
  iterate, relative to that last entry).
"""

import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from tests.gpu_helpers import assert_close, assert_hist_close, dev, f32, host, rel, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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
    assert_close(host(r.x), ref.x, 1e-4, "C2 BA k=2 x")
    assert_hist_close(r.res, ref.res, 1e-4, "C2 BA k=2")


def test_ba_gmres_50_iterations_match_the_oracle(c2):
    desc, g, b = c2
    say("C2 BA-GMRES(B_un) K = 50 against the oracle")
    r = ct.ct_ba_gmres(g, dev(b), 50)
    ref = oracle.ba_gmres(desc, b, 50)
    assert r.iters_done == ref.iters_done == 50
    assert_close(host(r.x), ref.x, 1e-4, "C2 BA K=50 x")
    assert_hist_close(r.res, ref.res, 1e-4, "C2 BA K=50")


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
    true = float(torch.linalg.vector_norm(rr.double()))
    say("C2 recomputed residual %.6e, carried %.6e" % (true, res[-1]))
    assert abs(true - res[-1]) <= 1e-2 * res[-1]


def _cgls_spread():
    with open(os.path.join(HERE, "golden", "cgls_fp32_spread.json")) as f:
        return json.load(f)["w2_cgls_AT_50"]


def test_cgls_AT_50_iterations_match_the_oracle(c2):
    desc, g, b = c2
    say("C2 CGLS(A^T) K = 50 against the oracle")
    r = ct.ct_cgls(g, dev(b), 50, B="AT")
    ref = oracle.cgls(desc, b, 50, B="AT")
    assert r.iters_done == ref.iters_done == 50
    spread = _cgls_spread()
    say("C2 CGLS(A^T) oracle FP32-vector spread: x %.3e, residual %.3e" % (spread["x"], spread["res"]))
    assert_hist_close(r.res, ref.res, max(1e-4, 3.0 * spread["res"]), "C2 CGLS(A^T) K=50")
    assert_close(host(r.x), ref.x, max(1e-4, 3.0 * spread["x"]), "C2 CGLS(A^T) K=50 x")


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
    say("C2 CGLS recomputed residual %.6e, carried %.6e" % (true, res[-1]))
    assert abs(true - res[-1]) <= 2e-2 * res[-1]
