"""GPU solver parity with the FP64 oracle.

Tolerance for reconstructions and residual histories at a fixed iteration
count: relative 1e-4.  Derivation: the operators agree to ~1e-6 (see the
operator tests); GMRES propagates operator perturbations through the
Krylov space with a growth set by the conditioning of the small Hessenberg
problem, which stays below 1e2 for k <= 50 on these workloads (measured);
the FP32 basis adds orthogonality loss of order 1e-7 per vector.
"""

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from synth.phantoms import random_ellipsoids, rasterize_ellipsoids
from synth.geometry import cone3d
from tests.gpu_helpers import assert_close, assert_hist_close, dev, f32, fp32_envelope, fp32_envelopes, host, rel, say

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def w1():
    desc = workloads.w1_geometry()
    x_true = workloads.w1_phantom()
    clean = oracle.project_A(desc, x_true)
    b = f32(clean + workloads.relative_gaussian_noise(clean, 0.01, 102))
    return desc, ct.Geometry(desc), b


@pytest.fixture(scope="module")
def cone_small():
    desc = cone3d(48, 60, 72)
    ells = random_ellipsoids(211, 8, 48.0)
    x_true = rasterize_ellipsoids(ells, 48, 1.0)
    b = f32(oracle.project_A(desc, f32(x_true)))
    return desc, ct.Geometry(desc), b


def _compare(res_gpu, ref, x_tol=TOL, what="", hist_tol=TOL):
    """Iterate: relative 2-norm and every voxel against the largest one;
    residual history: every entry relative to itself."""
    assert res_gpu.iters_done == ref.iters_done
    assert_close(host(res_gpu.x), ref.x, x_tol, what + " x")
    assert_hist_close(res_gpu.res, ref.res, hist_tol, what)


def _compare_in_envelope(res_gpu, ref, desc, b, K, B, solver, what):
    """Noisy data: the iterate's elements and each residual entry within
    three times the move that FP32-sized perturbations of the oracle's own
    operators cause (fp32_envelopes), and never looser than 1e-4; the
    iterate as a whole (relative 2-norm) within 1e-4 of the oracle's, the
    reconstruction accuracy asked of the FP32 path at a fixed iteration
    count (measured 2.6e-6 .. 3.8e-5 here)."""
    ex, er = fp32_envelopes(desc, b, K, B, solver)
    say("%s FP32 envelope: iterate %.3e, residual entries %.3e" % (what, ex, er))
    _compare(res_gpu, ref, max(TOL, 3.0 * ex), what, max(TOL, 3.0 * er))
    assert rel(host(res_gpu.x), ref.x) <= TOL, (what, rel(host(res_gpu.x), ref.x))


# On the noisy 64^2 problem FP32-sized perturbations of the oracle's own
# operators move the BA-GMRES iterate by up to 2.1e-4 at k = 15 and 1.1e-4
# at k = 30 (B_un, A^T; 9e-6 and 8e-5 with B_FBP), and its residual entries,
# which lie 1e2..1e4 below the first one, by up to 7.8e-3 at k = 15 and 18 %
# at k = 30 (mid-history entries, which recover by the last iteration).
# Both are held to three times the envelope measured on the spot, and the
# iterate's relative 2-norm distance to 1e-4 besides.
@pytest.mark.parametrize("B", ["un", "ramp", "AT"])
def test_ba_gmres_w1(w1, B):
    desc, g, b = w1
    say("BA-GMRES W1", B)
    for K in (15, 30):
        r = ct.ct_ba_gmres(g, dev(b), K, B=B)
        _compare_in_envelope(r, oracle.ba_gmres(desc, b, K, B=B), desc, b, K, B, "ba", "BA %s k=%d" % (B, K))


@pytest.mark.parametrize("B", ["un", "ramp"])
def test_ab_gmres_w1(w1, B):
    desc, g, b = w1
    say("AB-GMRES W1", B)
    for K in (15, 30):
        r = ct.ct_ab_gmres(g, dev(b), K, B=B)
        _compare_in_envelope(r, oracle.ab_gmres(desc, b, K, B=B), desc, b, K, B, "ab", "AB %s k=%d" % (B, K))


def test_cgls_AT_w1(w1):
    """CGLS is a short recurrence: rounding in the stored vectors is
    amplified from step to step.  Run in the oracle's own arithmetic with the
    vectors rounded to FP32, CGLS(A^T) on this workload differs from the FP64
    run by 2e-7 at k = 5, 1e-4 at k = 8 and 1.3e-2 at k = 10 (measured), so
    parity to 1e-4 is asserted up to k = 6; at k = 30 the data residual
    ||b - A x_30|| must agree to 2 % and x to 3 %."""
    desc, g, b = w1
    say("CGLS(A^T) W1")
    _compare(ct.ct_cgls(g, dev(b), 6, B="AT"), oracle.cgls(desc, b, 6, B="AT"), what="CGLS(A^T) k=6")
    r = ct.ct_cgls(g, dev(b), 30, B="AT")
    ref = oracle.cgls(desc, b, 30, B="AT")
    assert r.iters_done == 30
    assert abs(r.res[-1] - ref.res[-1]) <= 2e-2 * ref.res[-1]
    assert rel(host(r.x), ref.x) <= 3e-2
    assert np.all(np.diff(np.array(r.res)) <= 0.0)


def test_cgls_unmatched_w1_reported(w1):
    """CGLS with B_un has no convergence theory (parity unpinned in the
    oracle beyond its recurrence); GPU-vs-oracle agreement is asserted for the
    first iterations only, for the reason given above."""
    desc, g, b = w1
    r = ct.ct_cgls(g, dev(b), 6, B="un")
    _compare(r, oracle.cgls(desc, b, 6, B="un"), what="CGLS(B_un) k=6")


@pytest.mark.parametrize("B", ["un", "ramp"])
def test_ba_gmres_cone_small(cone_small, B):
    desc, g, b = cone_small
    say("BA-GMRES cone 48^3", B)
    r = ct.ct_ba_gmres(g, dev(b), 20, B=B)
    _compare(r, oracle.ba_gmres(desc, b, 20, B=B), what="BA cone 48^3 %s k=20" % B)


def test_ab_gmres_and_cgls_cone_small(cone_small):
    desc, g, b = cone_small
    say("AB-GMRES / CGLS cone 48^3")
    _compare(ct.ct_ab_gmres(g, dev(b), 12, B="un"), oracle.ab_gmres(desc, b, 12, B="un"), what="AB cone k=12")
    _compare(ct.ct_cgls(g, dev(b), 6, B="AT"), oracle.cgls(desc, b, 6, B="AT"), what="CGLS(A^T) cone k=6")


def test_ba_gmres_fp16_storage_w1(w1):
    """FP16 storage of the projections: reported tolerance (FP16 unit
    roundoff 4.9e-4), not held to the FP32 bound."""
    desc, g, b = w1
    r16 = ct.ct_ba_gmres(g, dev(b), 30, B="ramp", sino_dtype=torch.float16)
    ref = oracle.ba_gmres(desc, b, 30, B="ramp")
    e = rel(host(r16.x), ref.x)
    say("FP16-storage BA-GMRES W1 rel err", e)
    assert r16.iters_done == 30
    assert e <= 2e-2


def test_ba_gmres_full_w3_properties():
    """Headline workload (256^3 cone beam, ramp-filtered B, K = 30), the
    launch configuration the benchmark times.  The full FP64 solve is too
    slow for the oracle, so properties that hold at any size are checked:
    the residual history is non-increasing, its last entry equals the
    recomputed ||B b - B A x_K|| (with the GPU operators), and the first
    residual equals ||B b||."""
    desc = workloads.w3_geometry()
    say("W3 BA-GMRES properties")
    g = ct.Geometry(desc)
    vol = workloads.w3_phantom()
    b = ct.ct_project_A(g, dev(vol))
    r = ct.ct_ba_gmres(g, b.reshape(-1), 30, B="ramp")
    assert r.iters_done == 30
    res = np.array(r.res)
    assert np.all(np.diff(res) <= 1e-6 * res[0])
    Bb = ct.ct_backproject_B(g, b, ramp=True)
    assert abs(float(torch.linalg.vector_norm(Bb.double())) - res[0]) <= 1e-5 * res[0]
    Ax = ct.ct_project_A(g, r.x)
    rr = Bb - ct.ct_backproject_B(g, Ax, ramp=True)
    true = float(torch.linalg.vector_norm(rr.double()))
    say("W3 recomputed residual %.6e, carried %.6e" % (true, res[-1]))
    # relative to the last residual itself (a bound relative to res[0] would
    # be wider than res[-1] once the residual has fallen below it)
    assert abs(true - res[-1]) <= 2e-2 * res[-1]
