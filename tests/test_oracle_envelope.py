"""The FP32 envelope against real FP32 rounding orders (CPU, oracle only).

The GPU solvers on noisy data are held to three times the FP32 envelope
(`tests/gpu_helpers.fp32_envelope`): the largest move of the oracle's K-th
iterate when every operator output is perturbed by FP32-sized relative
noise.  Different FP32 summation orders of one operator are such
perturbations; the ramp filter F (Sec. III, B_FBP = B_un F) is the operator
whose order the GPU kernels have changed.  Here the oracle's BA-GMRES with
B = B_un F runs with F evaluated in FP32 with two summation orders (lags
ascending and lags descending, every product and partial sum rounded to
FP32) and everything else in FP64.  On the noisy 64^2 problem at K = 30
each order moves the iterate by a different amount, and both moves must
lie within three times the envelope the GPU tests use (for the Joseph and
the line-intersection forward models)."""

import numpy as np
import pytest

import oracle
from synth import workloads
from synth.geometry import parallel2d
from tests.gpu_helpers import fp32_envelope

K = 30


def _ramp_taps(desc):
    """The oracle's filter as taps h[lag], lag = -(nu-1) .. nu-1, read off
    its responses to unit impulses at the first and last bin of a row."""
    nu = desc.nu
    taps = np.zeros(2 * nu - 1)
    for k in (0, nu - 1):
        e = np.zeros(desc.sino_shape)
        e.reshape(-1, nu)[0, k] = 1.0
        out = np.asarray(oracle.ramp(desc, e)).reshape(-1, nu)[0]
        for j in range(nu):
            taps[(j - k) + nu - 1] = out[j]
    return taps


def _ramp32(q, taps, nu, ascending):
    """out[j] = sum over lags l of taps[l] q[j - l] within each row, every
    product and partial sum rounded to FP32, lags in the given order."""
    rows = np.asarray(q, np.float64).reshape(-1, nu).astype(np.float32)
    t32 = taps.astype(np.float32)
    acc = np.zeros_like(rows)
    lags = range(-(nu - 1), nu) if ascending else range(nu - 1, -nu, -1)
    for l in lags:
        h = t32[l + nu - 1]
        if h == 0.0:
            continue
        sh = np.zeros_like(rows)
        if l >= 0:
            sh[:, l:] = rows[:, :nu - l]
        else:
            sh[:, :nu + l] = rows[:, -l:]
        acc = (acc + (h * sh).astype(np.float32)).astype(np.float32)
    return acc.astype(np.float64).reshape(-1)


@pytest.mark.parametrize("projector", [0, 1])
def test_ramp_rounding_orders_inside_fp32_envelope(projector):
    desc = parallel2d(64, 90, 96, projector=projector)
    clean = np.asarray(oracle.project_A(desc, workloads.w1_phantom()))
    b = (clean + workloads.relative_gaussian_noise(clean, 0.01, 102)).astype(np.float32).astype(np.float64)
    ref = np.asarray(oracle.ba_gmres(desc, b, K, B="ramp").x).reshape(-1)
    env = fp32_envelope(desc, b, K, B="ramp")
    taps = _ramp_taps(desc)
    # the taps reproduce the oracle's filter in FP64
    q = np.random.default_rng(1).standard_normal(desc.n_rays)
    rows = q.reshape(-1, desc.nu)
    conv = np.stack([np.convolve(r, taps)[desc.nu - 1:2 * desc.nu - 1] for r in rows]).reshape(-1)
    assert np.allclose(conv, np.asarray(oracle.ramp(desc, q)), rtol=0, atol=1e-12 * np.abs(conv).max())

    A = lambda v: np.asarray(oracle.project_A(desc, v.reshape(desc.vol_shape))).reshape(-1)
    Bun = lambda y: np.asarray(oracle.backproject_Bun(desc, y.reshape(desc.sino_shape))).reshape(-1)
    moves = []
    for ascending in (True, False):
        F = lambda y: _ramp32(y, taps, desc.nu, ascending)
        co, W, res, done, _ = oracle.gmres(lambda v: Bun(F(A(v))), Bun(F(b)), K)
        assert done == K
        x = W[:done].T @ co
        moves.append(float(np.linalg.norm(x - ref) / np.linalg.norm(ref)))
    print("projector %d: FP32 ramp orders move x_%d by %.3e (ascending) and %.3e (descending); "
          "FP32 envelope %.3e" % (projector, K, moves[0], moves[1], env))
    assert moves[0] != moves[1]               # two distinct rounding orders
    assert max(moves) <= 3.0 * env, (moves, env)
