"""Pins of the oracle's solvers (Sec. II of the paper) against textbook
equivalences, finite termination, brute force and invariants.

* BA-GMRES with B = A^T minimises ||A^T (b - A x)|| over K_k(A^T A, A^T b),
  which is exactly LSMR's iterate k (scipy's LSMR, no damping or stopping).
* AB-GMRES with B = A^T and CGLS with B = A^T minimise ||b - A x|| over the
  same space: LSQR's iterate k.
* At k = n, BA-GMRES solves B A x = B b (dense solve); at k = m <= n,
  AB-GMRES gives A x = b.
* For small k, x_k is the least-squares minimiser of ||B(b - A x)|| over an
  explicit Krylov matrix.
* The recorded residual is non-increasing (the method minimises it) and equals
  the recomputed ||B b - B A x_k||.
"""

import numpy as np
import pytest
from scipy.sparse.linalg import LinearOperator, lsmr, lsqr

from synth.geometry import parallel2d
from synth import workloads


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def w1(oracle):
    g = workloads.w1_geometry()
    x_true = workloads.w1_phantom()
    clean = oracle.project_A(g, x_true)
    b = clean + workloads.relative_gaussian_noise(clean, 0.01, 102)
    return g, x_true, b


def _linop(oracle, g):
    return LinearOperator((g.n_rays, g.n_vox), matvec=lambda v: oracle.project_A(g, v),
                          rmatvec=lambda w: oracle.backproject_AT(g, w), dtype=np.float64)


@pytest.mark.parametrize("k", [1, 4, 8])
def test_ba_gmres_with_AT_equals_lsmr(oracle, w1, k):
    g, _, b = w1
    r = oracle.ba_gmres(g, b, k, B="AT")
    xl = lsmr(_linop(oracle, g), b, damp=0.0, atol=0, btol=0, conlim=0, maxiter=k)[0]
    assert r.iters_done == k
    assert rel(r.x, xl) <= 1e-9


@pytest.mark.parametrize("k", [1, 4, 8])
def test_ab_gmres_and_cgls_with_AT_equal_lsqr(oracle, w1, k):
    g, _, b = w1
    xl = lsqr(_linop(oracle, g), b, damp=0.0, atol=0, btol=0, conlim=0, iter_lim=k)[0]
    ra = oracle.ab_gmres(g, b, k, B="AT")
    rc = oracle.cgls(g, b, k, B="AT")
    assert rel(ra.x, xl) <= 1e-9
    assert rel(rc.x, xl) <= 1e-9
    # CGLS's recursive residual is ||b - A x_k||
    assert abs(rc.res[-1] - np.linalg.norm(b - oracle.project_A(g, rc.x))) <= 1e-8 * rc.res[-1]


@pytest.mark.parametrize("k", [12, 20, 30])
def test_gmres_with_AT_not_worse_than_short_recurrences(oracle, w1, k):
    """Past a few steps LSMR and LSQR lose orthogonality in FP64 on this
    ill-conditioned problem while GMRES keeps an orthonormal basis, so only
    optimality is asserted: GMRES's objective is no larger than theirs."""
    g, _, b = w1
    L = _linop(oracle, g)
    xm = lsmr(L, b, damp=0.0, atol=0, btol=0, conlim=0, maxiter=k)[0]
    xq = lsqr(L, b, damp=0.0, atol=0, btol=0, conlim=0, iter_lim=k)[0]
    ba = oracle.ba_gmres(g, b, k, B="AT").x
    ab = oracle.ab_gmres(g, b, k, B="AT").x
    fba = lambda x: np.linalg.norm(oracle.backproject_AT(g, b - oracle.project_A(g, x)))
    fab = lambda x: np.linalg.norm(b - oracle.project_A(g, x))
    assert fba(ba) <= fba(xm) * (1 + 1e-12)
    assert fab(ab) <= fab(xq) * (1 + 1e-12)


def _dense(oracle, g):
    n, m = g.n_vox, g.n_rays
    A = np.stack([oracle.project_A(g, np.eye(n)[j]) for j in range(n)], axis=1)
    Bun = np.stack([oracle.backproject_Bun(g, np.eye(m)[i]) for i in range(m)], axis=1)
    return A, Bun


def test_ba_gmres_finite_termination_k_equals_n(oracle):
    g = parallel2d(16, 24, 24)
    A, B = _dense(oracle, g)
    rng = np.random.default_rng(12)
    b = A @ rng.uniform(size=256) + 0.01 * rng.standard_normal(g.n_rays)
    S = B @ A
    cond = np.linalg.cond(S)
    x_ref = np.linalg.solve(S, B @ b)
    r = oracle.ba_gmres(g, b, 256, B="un")
    assert r.iters_done <= 256
    assert rel(r.x, x_ref) <= 1e-15 * cond, cond


def test_ba_gmres_ramp_finite_termination_k_equals_n(oracle):
    """With B = B_un F (the ramp-filtered back-projector, Sec. III) and B A
    nonsingular, BA-GMRES at k = n solves B A x = B b exactly: the dense
    system built column by column from unit vectors decides the iterate."""
    g = parallel2d(16, 24, 24)
    n, m = g.n_vox, g.n_rays
    A = np.stack([oracle.project_A(g, np.eye(n)[j]) for j in range(n)], axis=1)
    Bf = oracle.back_projector(g, "ramp")
    B = np.stack([Bf(np.eye(m)[i]) for i in range(m)], axis=1)
    rng = np.random.default_rng(15)
    b = A @ rng.uniform(size=n) + 0.01 * rng.standard_normal(m)
    S = B @ A
    cond = np.linalg.cond(S)
    x_ref = np.linalg.solve(S, B @ b)
    r = oracle.ba_gmres(g, b, n, B="ramp")
    assert r.iters_done <= n
    assert rel(r.x, x_ref) <= 1e-15 * cond, cond


def test_ab_gmres_finite_termination_k_equals_m(oracle):
    """With m <= n and A B nonsingular, AB-GMRES at k = m solves A x = b.
    The detector is narrower than the image and the angles avoid 0/90 deg,
    so no two views share a total-sum row dependency."""
    import math
    g = parallel2d(16, 6, 12, angles=[(p + 0.3) * math.pi / 6 for p in range(6)])
    A, B = _dense(oracle, g)
    assert np.linalg.matrix_rank(A @ B) == g.n_rays
    cond = np.linalg.cond(A @ B)
    rng = np.random.default_rng(13)
    b = rng.standard_normal(g.n_rays)
    r = oracle.ab_gmres(g, b, g.n_rays, B="un")
    assert rel(oracle.project_A(g, r.x), b) <= 1e-15 * cond, cond


@pytest.mark.parametrize("B", ["un", "ramp"])
def test_ba_gmres_brute_force_krylov(oracle, B):
    g = parallel2d(16, 20, 24)
    rng = np.random.default_rng(14)
    b = rng.standard_normal(g.n_rays)
    Bop = oracle.back_projector(g, B)
    Bb = Bop(b)
    for k in range(1, 7):
        K = [Bb]
        for _ in range(k - 1):
            K.append(Bop(oracle.project_A(g, K[-1])))
        K = np.stack(K, axis=1)
        K = K / np.linalg.norm(K, axis=0)
        BAK = np.stack([Bop(oracle.project_A(g, K[:, j])) for j in range(k)], axis=1)
        c = np.linalg.lstsq(BAK, Bb, rcond=None)[0]
        r = oracle.ba_gmres(g, b, k, B=B)
        assert rel(r.x, K @ c) <= 1e-8


@pytest.mark.parametrize("B", ["un", "ramp"])
def test_ba_gmres_residual_monotone_and_true(oracle, w1, B):
    g, _, b = w1
    Bop = oracle.back_projector(g, B)
    Bb = Bop(b)
    r = oracle.ba_gmres(g, b, 30, B=B, keep_basis=True)
    res = np.array(r.res)
    assert res[0] == pytest.approx(np.linalg.norm(Bb), rel=1e-15)
    assert np.all(np.diff(res) <= 1e-14 * res[0])
    true_res = np.linalg.norm(Bb - Bop(oracle.project_A(g, r.x)))
    assert abs(true_res - res[-1]) <= 1e-10 * res[0]
    # first basis vector is B b / ||B b|| and the basis is orthonormal
    assert np.array_equal(r.W[0], Bb / np.linalg.norm(Bb))
    G = r.W @ r.W.T
    assert np.max(np.abs(G - np.eye(G.shape[0]))) <= 1e-12


def test_ab_gmres_residual_is_data_residual(oracle, w1):
    g, _, b = w1
    r = oracle.ab_gmres(g, b, 20, B="un")
    res = np.array(r.res)
    assert np.all(np.diff(res) <= 1e-14 * res[0])
    assert abs(np.linalg.norm(b - oracle.project_A(g, r.x)) - res[-1]) <= 1e-10 * res[0]


def test_ba_gmres_power_of_two_scale_invariance(oracle, w1):
    g, _, b = w1
    Bop = oracle.back_projector(g, "un")
    A = lambda v: oracle.project_A(g, v)
    c1, W1, res1, k1, _ = oracle.gmres(lambda v: Bop(A(v)), Bop(b), 15)
    c2, W2, res2, k2, _ = oracle.gmres(lambda v: 2.0 * Bop(A(v)), 2.0 * Bop(b), 15)
    assert k1 == k2 == 15
    assert np.array_equal(W1.T @ c1, W2.T @ c2)
    assert np.array_equal(2.0 * np.array(res1), np.array(res2))


def test_zero_rhs_and_happy_breakdown(oracle):
    g = parallel2d(16, 12, 24)
    r = oracle.ba_gmres(g, np.zeros(g.n_rays), 10)
    assert r.iters_done == 0 and np.all(r.x == 0) and r.res == [0.0]
    # one pixel, one view, one bin: B A is 1x1 and the first step is exact
    g1 = parallel2d(1, 1, 1)
    r1 = oracle.ba_gmres(g1, np.array([2.5]), 5)
    assert r1.iters_done == 1
    a = oracle.project_A(g1, np.array([1.0]))[0]
    assert r1.x[0] == pytest.approx(2.5 / a, rel=1e-15)
    assert r1.res[-1] <= 1e-15


def test_cgls_with_unmatched_B_runs(oracle, w1):
    """CGLS with B_un has no convergence theory; only that it runs and that
    its recursive residual tracks ||b - A x_k|| is checked (parity unpinned
    beyond this)."""
    g, _, b = w1
    rc = oracle.cgls(g, b, 30, B="un")
    assert rc.iters_done == 30
    assert abs(rc.res[-1] - np.linalg.norm(b - oracle.project_A(g, rc.x))) <= 1e-6 * rc.res[0]
