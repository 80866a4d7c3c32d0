"""The headline 256^3 cone-beam workload (360 views of a 384 x 384 detector,
ellipsoids plus texture, Poisson data at 1e5 photons, negative log) at its
full size, in the launch configuration the benchmark times: BA-GMRES with
the ramp-filtered back-projector B_FBP = B_un F (Sec. II, Eq. 5; Sec. III)
against the FP64 oracle, iterate and residual history.

The data come from the oracle's projector (FP64, rounded once to FP32), so
a defect of the GPU's A cannot shape the right-hand side both sides solve.
The oracle takes about 20 s per iteration at this size on the host's
threads, so K = 3: few enough iterations that FP32 operators cannot move
the exact iterate by more than ~1e-6 (the perturbation growth that forces
an envelope on noisy data appears only after tens of iterations), so the
iterate is held to 1e-4 in the 2-norm and per voxel, and every residual
entry to 1e-4 of itself."""

import numpy as np
import pytest

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from synth.phantoms import poisson_log_counts
from tests.gpu_helpers import assert_close, assert_hist_close, dev, host, say

pytestmark = pytest.mark.gpu

K = 3


@pytest.fixture(scope="module")
def c3():
    desc = workloads.w3_geometry()
    say("C3 data from the oracle's projector")
    vol = workloads.w3_phantom()
    clean = np.asarray(oracle.project_A(desc, vol))
    mu = 4.0 / float(clean.max())
    b = poisson_log_counts(303, clean * mu, 1e5).astype(np.float32)
    return desc, ct.Geometry(desc), b


def test_headline_workload_data(c3):
    desc, g, b = c3
    assert b.shape == (desc.n_rays,)
    # line integrals up to 4 plus Poisson noise; rays through air can count
    # more than the incident photons, so b dips slightly below zero
    assert np.all(np.isfinite(b)) and 3.5 < float(b.max()) < 4.5 and float(b.min()) > -0.1


def test_ba_gmres_ramp_matches_the_oracle(c3):
    desc, g, b = c3
    say("C3 BA-GMRES(B_FBP) K = %d on the GPU" % K)
    r = ct.ct_ba_gmres(g, dev(b), K, B="ramp")
    x = host(r.x)
    say("C3 BA-GMRES(B_FBP) K = %d in the oracle" % K)
    ref = oracle.ba_gmres(desc, b.astype(np.float64), K, B="ramp")
    assert r.iters_done == ref.iters_done == K
    assert_close(x, ref.x, 1e-4, "C3 BA(B_FBP) K=%d x" % K)
    assert_hist_close(r.res, ref.res, 1e-4, "C3 BA(B_FBP) K=%d" % K)
