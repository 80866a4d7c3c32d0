"""Restarted BA-GMRES(m) (ct_ba_gmres_restarted) against the oracle's
restarted loop, and its first cycle against the unrestarted solver.

A later cycle starts from the data residual b - A x, about a hundred times
smaller than b here, so an iterate within 1e-5 of the oracle's gives a
residual within ~1e-3 of the oracle's, relative to itself.  The residual
histories are therefore compared on the scale of the first cycle's start
||B b|| (1e-4 of it), the iterates at 1e-4 as for the other solvers."""

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from synth.geometry import cone3d
from tests.gpu_helpers import dev, f32, host, rel, say

pytestmark = pytest.mark.gpu

TOL = 1e-4


def w1_data():
    desc = workloads.w1_geometry()
    x_true = workloads.w1_phantom()
    clean = oracle.project_A(desc, x_true)
    return desc, f32(clean + workloads.relative_gaussian_noise(clean, 0.01, 102))


def test_one_cycle_is_the_plain_solver():
    desc, b = w1_data()
    g = ct.Geometry(desc)
    r = ct.ct_ba_gmres_restarted(g, dev(b), 12, 1)
    p = ct.ct_ba_gmres(g, dev(b), 12)
    assert torch.equal(r.x, p.x) and r.res[0] == p.res and r.iters_done == p.iters_done


@pytest.mark.parametrize("B", ["un", "ramp"])
def test_restarted_2d_matches_oracle(B):
    desc, b = w1_data()
    g = ct.Geometry(desc)
    say("restarted 2d", B)
    r = ct.ct_ba_gmres_restarted(g, dev(b), 10, 3, B=B)
    x_ref, hist = oracle.ba_gmres_restarted(desc, b, 10, 3, B=B)
    assert r.iters_done == 30
    assert rel(host(r.x), x_ref) <= TOL
    scale = hist[0][0]
    for c in range(3):
        assert np.max(np.abs(np.array(r.res[c]) - np.array(hist[c]))) <= TOL * scale, c
    # each cycle starts where the previous one ended (same B-residual)
    assert abs(r.res[1][0] - r.res[0][-1]) <= 1e-3 * r.res[0][-1]


def test_restarted_cone_matches_oracle():
    desc = cone3d(32, 30, 48)
    g = ct.Geometry(desc)
    b = f32(oracle.project_A(desc, workloads.w2_phantom(n=32)))
    r = ct.ct_ba_gmres_restarted(g, dev(b), 6, 2, B="ramp")
    x_ref, hist = oracle.ba_gmres_restarted(desc, b, 6, 2, B="ramp")
    assert rel(host(r.x), x_ref) <= TOL
    assert np.max(np.abs(np.array(r.res[1]) - np.array(hist[1]))) <= TOL * hist[0][0]
