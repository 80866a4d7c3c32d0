"""Pins of the oracle's FP16 storage of the GMRES basis.

The paper names the stored basis (one vector per iteration) as the method's
memory burden (Sec. II).  Storing each vector in FP16 is this
implementation's option, not the paper's; the oracle defines it as the FP64
algorithm with every stored basis vector replaced by its FP16 rounding
(after a power-of-two scale that puts its values near 1).  The pins check it
against what that definition fixes:

* rounding happens and is bounded by FP16's unit roundoff: the basis is
  unit-norm and orthonormal to within a few 2^-11, but not exactly;
* the iterate stays within the FP16 rounding level of the FP64-basis
  iterate and the residual history follows it;
* a power-of-two scaling of the right-hand side scales the result exactly
  (the stored values do not change), also at magnitudes where unscaled
  FP16 storage would overflow or flush to zero;
* the scale choice puts t * norm in (sqrt(n)/2, sqrt(n)].
"""

import math

import numpy as np
import pytest

from synth import workloads

U16 = 2.0 ** -11     # FP16 unit roundoff


def _dense_problem(n=60, seed=5):
    rng = np.random.default_rng(seed)
    M = np.eye(n) + 0.4 * rng.standard_normal((n, n)) / math.sqrt(n)
    r0 = rng.standard_normal(n)
    return M, r0


def test_basis_rounded_but_orthonormal_to_fp16_level(oracle):
    M, r0 = _dense_problem()
    co, W, res, done, _ = oracle.gmres(lambda v: M @ v, r0, 20, basis="f16")
    assert done == 20
    G = W @ W.T
    off = np.abs(G - np.eye(done))
    assert off.max() <= 8 * U16          # orthonormal to FP16 precision
    assert off.max() >= 1e-9             # ... and no better: the rounding is applied
    norms = np.linalg.norm(W, axis=1)
    assert np.all(np.abs(norms - 1.0) <= 4 * U16)


def test_iterate_follows_fp64_basis(oracle):
    M, r0 = _dense_problem()
    c64, W64, res64, d64, _ = oracle.gmres(lambda v: M @ v, r0, 15)
    c16, W16, res16, d16, _ = oracle.gmres(lambda v: M @ v, r0, 15, basis="f16")
    x64, x16 = W64.T @ c64, W16.T @ c16
    d = np.linalg.norm(x16 - x64) / np.linalg.norm(x64)
    assert 1e-9 <= d <= 2e-3
    # the residual recurrence: equal start, and each step within the rounding level
    assert res16[0] == res64[0]
    assert np.allclose(res16, res64, rtol=2e-3, atol=0)
    # the recorded residual is the true residual of the iterate to FP16 level
    true = np.linalg.norm(r0 - M @ x16)
    assert abs(true - res16[-1]) <= 4e-3 * res16[0]


@pytest.mark.parametrize("e", [-300, -60, 0, 60, 300])
def test_power_of_two_scale_is_exact(oracle, e):
    """2^e b gives exactly 2^e x: the stored FP16 values do not depend on
    the magnitude (2^300 overflows FP16 by far, 2^-60 underflows it)."""
    M, r0 = _dense_problem(n=40, seed=9)
    c1, W1, res1, _, _ = oracle.gmres(lambda v: M @ v, r0, 10, basis="f16")
    s = 2.0 ** e
    c2, W2, res2, _, _ = oracle.gmres(lambda v: M @ v, s * r0, 10, basis="f16")
    assert np.array_equal(W1, W2)
    assert np.array_equal(W1.T @ c1 * s, W2.T @ c2)
    assert np.all(np.isfinite(W2))


def test_one_large_entry_does_not_overflow(oracle):
    """All the norm in one entry: the stored value is t * ||v|| <= sqrt(n),
    far below FP16's largest finite value."""
    n = 4096
    r0 = np.zeros(n)
    r0[17] = 3.0e6
    r0[18] = 1.0
    co, W, res, done, _ = oracle.gmres(lambda v: 2.0 * v + np.roll(v, 1), r0, 4, basis="f16")
    assert np.all(np.isfinite(W)) and done == 4


def test_scale_choice(oracle):
    rng = np.random.default_rng(3)
    for n in (5, 4096, 16777216):
        for norm in 10.0 ** rng.uniform(-30, 30, size=50):
            t = oracle._pow2_below(norm, n)
            assert math.log2(t) == round(math.log2(t))
            assert math.sqrt(n) / 2 < t * norm <= math.sqrt(n)


@pytest.fixture(scope="module")
def w1_noisy(oracle):
    g = workloads.w1_geometry()
    x_true = workloads.w1_phantom()
    clean = oracle.project_A(g, x_true)
    return g, x_true.reshape(-1), clean + workloads.relative_gaussian_noise(clean, 0.01, 102)


def test_ba_gmres_fp16_basis_early_iterates(oracle, w1_noisy):
    """BA-GMRES on the 64 x 64 parallel-beam case, 5 iterations: the
    FP16-basis iterate is within the FP16 rounding level of the FP64-basis
    one and so is the residual history."""
    g, _, b = w1_noisy
    r64 = oracle.ba_gmres(g, b, 5)
    r16 = oracle.ba_gmres(g, b, 5, basis="f16")
    d = np.linalg.norm(r16.x - r64.x) / np.linalg.norm(r64.x)
    assert 1e-9 <= d <= 1e-2
    assert np.allclose(r16.res, r64.res, rtol=2e-3, atol=0)


def test_fp16_basis_floor_and_restart_recovery(oracle, w1_noisy):
    """Unrestarted, the rounding of the basis limits how far the residual
    falls (at 30 iterations it stays well above the FP64-basis one); with
    restarts every 10 iterations each cycle starts from the true residual
    and the FP16-basis result matches the FP64-basis one (image error within
    1 %, iterate within 1e-2)."""
    g, x_true, b = w1_noisy
    r64 = oracle.ba_gmres(g, b, 30)
    r16 = oracle.ba_gmres(g, b, 30, basis="f16")
    assert r16.res[-1] > 1.5 * r64.res[-1]
    x64, _ = oracle.ba_gmres_restarted(g, b, 10, 3)
    x16, _ = oracle.ba_gmres_restarted(g, b, 10, 3, basis="f16")
    e64 = np.linalg.norm(x64 - x_true) / np.linalg.norm(x_true)
    e16 = np.linalg.norm(x16 - x_true) / np.linalg.norm(x_true)
    assert abs(e16 - e64) <= 0.01 * e64
    assert np.linalg.norm(x16 - x64) / np.linalg.norm(x64) <= 1e-2
