"""Pins of the oracle's restarted BA-GMRES(m), the storage-bounding variant
the paper names for the Krylov basis (Sec. II).

Each cycle minimises ||B (r - A d)|| over K_m(BA, B r) for the data residual
r = b - A x of the current iterate and sets x <- x + d.  Hence the true
preconditioned residual at the start of a cycle equals the last residual
the previous cycle's rotations reported; with m equal to the image size one
cycle is the exact solve of B A x = B b; with B = A^T the cycles converge
to the least-squares solution.  The dense matrices come from the oracle's
operators, applied column by column (the operators are pinned elsewhere;
these pins are of the restart loop)."""

import numpy as np
import pytest

from synth.geometry import parallel2d, cone3d


def dense(oracle, g, fn, n_in, shape):
    cols = []
    for j in range(n_in):
        e = np.zeros(n_in)
        e[j] = 1.0
        cols.append(np.asarray(fn(g, e.reshape(shape))).reshape(-1))
    return np.stack(cols, axis=1)


def problem(seed=3):
    g = parallel2d(8, 16, 14)
    rng = np.random.default_rng(seed)
    x = rng.uniform(size=g.vol_shape)
    return g, x


@pytest.mark.parametrize("B", ["un", "ramp", "AT"])
def test_cycles_continue_each_others_residual(oracle, B):
    g, x_true = problem()
    b = np.asarray(oracle.project_A(g, x_true)).reshape(-1)
    b = b + 0.01 * np.linalg.norm(b) / np.sqrt(b.size) * np.random.default_rng(5).normal(size=b.size)
    x, hist = oracle.ba_gmres_restarted(g, b, 5, 6, B=B)
    Bop = oracle.back_projector(g, B)
    for c in range(len(hist)):
        h = np.array(hist[c])
        assert np.all(np.diff(h) <= 1e-12 * h[0]), (c, h)
        if c + 1 < len(hist):
            assert abs(hist[c + 1][0] - hist[c][-1]) <= 1e-10 * hist[0][0], (c, hist[c][-1], hist[c + 1][0])
    r = b - np.asarray(oracle.project_A(g, x.reshape(g.vol_shape))).reshape(-1)
    assert abs(np.linalg.norm(np.asarray(Bop(r.reshape(g.sino_shape)))) - hist[-1][-1]) <= 1e-10 * hist[0][0]
    assert hist[-1][-1] < 0.5 * hist[0][-1]


def test_full_length_cycle_is_the_exact_solve(oracle):
    g, x_true = problem()
    A = dense(oracle, g, oracle.project_A, g.n_vox, g.vol_shape)
    Bm = dense(oracle, g, oracle.backproject_Bun, g.n_rays, g.sino_shape)
    b = A @ x_true.reshape(-1) + np.random.default_rng(6).normal(scale=0.05, size=g.n_rays)
    x, hist = oracle.ba_gmres_restarted(g, b, g.n_vox, 1, B="un")
    ref = np.linalg.solve(Bm @ A, Bm @ b)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


def test_with_AT_converges_to_least_squares(oracle):
    g = cone3d(4, 10, 8, nz=3, nv=4)
    x_true = np.random.default_rng(8).uniform(size=g.vol_shape)
    A = dense(oracle, g, oracle.project_A, g.n_vox, g.vol_shape)
    b = A @ x_true.reshape(-1) + np.random.default_rng(9).normal(scale=0.05, size=g.n_rays)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    x, hist = oracle.ba_gmres_restarted(g, b, 16, 40, B="AT")
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref), np.linalg.norm(x - ref) / np.linalg.norm(ref)
    # a restart that subtracted its correction, or that restarted from b
    # instead of the residual, would not reach this point
