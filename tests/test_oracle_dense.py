"""Brute-force pins on tiny problems: the oracle's A against a dense matrix
built by a second route, its A^T against that matrix's transpose, and its
ramp filter against an FFT convolution.

The second route for A writes each matrix entry from the definition of
Joseph's method as a sum of tent functions: on the plane through voxel
centre i_a of the dominant axis a, the ray passes through the continuous
in-plane index f, and voxel (i_a, i_b[, i_c]) receives
    Delta / |d_a| * tent(f_b - i_b) [* tent(f_c - i_c)],  tent(t) = max(0, 1 - |t|)
for a unit direction d.  The oracle instead walks planes and splits a floor
and a fraction; the two agree only if plane positions, index offsets, the
dominant-axis choice, the step weight and the zero-outside rule all match.
Rays come from tests/analytic.py (source, detector centre and axes built
with vector algebra).
"""

import math

import numpy as np
import pytest

from synth.geometry import parallel2d, cone3d
from tests import analytic


def tent(t):
    return np.maximum(0.0, 1.0 - np.abs(t))


def dense_A_2d(g):
    O, D = analytic.rays_2d(g)
    th = analytic.angles_of(g)
    n = g.nx
    centres = (np.arange(n) - 0.5 * (n - 1)) * g.voxel
    A = np.zeros((g.n_views * g.nu, n * n))
    for p in range(g.n_views):
        if g.angles is None:
            xmajor = g.n_views <= 4 * p <= 3 * g.n_views
        else:
            xmajor = abs(math.sin(th[p])) >= abs(math.cos(th[p]))
        a, b = (0, 1) if xmajor else (1, 0)
        for k in range(g.nu):
            o, d = O[p, k], D[p, k]
            row = np.zeros((n, n))                      # [iy][ix]
            for i in range(n):
                t = (centres[i] - o[a]) / d[a]
                f = (o[b] + t * d[b]) / g.voxel + 0.5 * (n - 1)
                w = g.voxel / abs(d[a]) * tent(f - np.arange(n))
                if xmajor:
                    row[:, i] += w
                else:
                    row[i, :] += w
            A[p * g.nu + k] = row.reshape(-1)
    return A


def dense_A_cone(g):
    O, D = analytic.rays_3d(g)
    nx, ny, nz = g.nx, g.ny, g.nz
    cx = (np.arange(nx) - 0.5 * (nx - 1)) * g.voxel
    cy = (np.arange(ny) - 0.5 * (ny - 1)) * g.voxel
    A = np.zeros((g.n_rays, nz * ny * nx))
    r = 0
    for p in range(g.n_views):
        for v in range(g.nv):
            for u in range(g.nu):
                o, d = O[p, v, u], D[p, v, u]
                vol = np.zeros((nz, ny, nx))
                if abs(d[0]) >= abs(d[1]):
                    for i in range(nx):
                        t = (cx[i] - o[0]) / d[0]
                        fy = (o[1] + t * d[1]) / g.voxel + 0.5 * (ny - 1)
                        fz = (o[2] + t * d[2]) / g.voxel + 0.5 * (nz - 1)
                        vol[:, :, i] += (g.voxel / abs(d[0])) * np.outer(
                            tent(fz - np.arange(nz)), tent(fy - np.arange(ny)))
                else:
                    for i in range(ny):
                        t = (cy[i] - o[1]) / d[1]
                        fx = (o[0] + t * d[0]) / g.voxel + 0.5 * (nx - 1)
                        fz = (o[2] + t * d[2]) / g.voxel + 0.5 * (nz - 1)
                        vol[:, i, :] += (g.voxel / abs(d[1])) * np.outer(
                            tent(fz - np.arange(nz)), tent(fx - np.arange(nx)))
                A[r] = vol.reshape(-1)
                r += 1
    return A


def oracle_dense(oracle, g, fn, n_in):
    cols = []
    for j in range(n_in):
        e = np.zeros(n_in)
        e[j] = 1.0
        cols.append(np.asarray(fn(g, e.reshape(-1))).reshape(-1))
    return np.stack(cols, axis=1)


GEOMS_2D = {
    "16px_24views_24bins": parallel2d(16, 24, 24),
    "16px_24views_odd_pitch": parallel2d(16, 24, 23, du=0.8),
    "15px_explicit_angles": parallel2d(15, 5, 22, voxel=1.3, du=1.1,
                                       angles=[0.1, 0.7, 1.9, 2.5, 3.0]),
}


@pytest.mark.parametrize("name", list(GEOMS_2D))
def test_dense_A_and_AT_2d(oracle, name):
    g = GEOMS_2D[name]
    ref = dense_A_2d(g)
    n = g.n_vox
    A = oracle_dense(oracle, g, lambda gg, e: oracle.project_A(gg, e.reshape(g.vol_shape)), n)
    assert np.max(np.abs(A - ref)) <= 1e-14 * np.abs(ref).max()
    AT = oracle_dense(oracle, g, lambda gg, e: oracle.backproject_AT(gg, e.reshape(g.sino_shape)),
                      g.n_rays)
    assert np.max(np.abs(AT - ref.T)) <= 1e-14 * np.abs(ref).max()


def test_dense_A_and_AT_cone(oracle):
    g = cone3d(10, 6, 9, nz=8, nv=7, pitch=1.7, sod_factor=3.0, sdd_factor=5.0,
               angles=[0.2, 0.9, 1.6, 2.8, 4.0, 5.5])
    ref = dense_A_cone(g)
    A = oracle_dense(oracle, g, lambda gg, e: oracle.project_A(gg, e.reshape(g.vol_shape)), g.n_vox)
    assert np.max(np.abs(A - ref)) <= 1e-13 * np.abs(ref).max()
    AT = oracle_dense(oracle, g, lambda gg, e: oracle.backproject_AT(gg, e.reshape(g.sino_shape)),
                      g.n_rays)
    assert np.max(np.abs(AT - ref.T)) <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("nu,du", [(24, 1.0), (37, 0.45)])
def test_ramp_equals_zero_padded_fft_convolution(oracle, nu, du):
    """Linear (not circular) convolution with the Ram-Lak taps, computed by a
    zero-padded FFT; catches a circular wrap, a one-bin shift or a missing
    du factor."""
    g = parallel2d(8, 3, nu, du=du)
    q = np.random.default_rng(5).normal(size=g.sino_shape)
    lags = np.arange(-(nu - 1), nu)
    h = np.where(lags == 0, 1.0 / (4.0 * du * du),
                 np.where(lags % 2 != 0, -1.0 / (math.pi ** 2 * np.maximum(lags * lags, 1) * du * du), 0.0))
    L = 1
    while L < 3 * nu:
        L *= 2
    Hf = np.fft.rfft(h, L)
    ref = np.empty_like(q)
    for p in range(g.n_views):
        conv = np.fft.irfft(np.fft.rfft(q[p, 0], L) * Hf, L)
        ref[p, 0] = du * conv[nu - 1:2 * nu - 1]
    out = np.asarray(oracle.ramp(g, q)).reshape(q.shape)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.abs(ref).max()
