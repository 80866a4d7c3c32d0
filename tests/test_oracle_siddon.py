"""Pins of the oracle's line-intersection (Siddon) projector, the forward
model the paper uses (Sec. III): A_ij is the length of ray i inside voxel j.

The second route writes each entry by clipping the ray against voxel j's
own box (the slab method applied to one voxel), independently of the
oracle's sorted list of boundary crossings; the constant image gives the
chord through the whole grid; at 0 and 90 degrees the 2D rays run along
pixel columns and rows.  Rays come from tests/analytic.py.
"""

import numpy as np
import pytest

from synth.geometry import parallel2d, cone3d
from synth import phantoms
from tests import analytic


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def clip_length(o, d, lo, hi):
    """Length of the unit-speed line o + t d inside the box [lo, hi]."""
    t0, t1 = -np.inf, np.inf
    for a in range(len(o)):
        if d[a] == 0.0:
            if not (lo[a] < o[a] < hi[a]):
                return 0.0
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return max(t1 - t0, 0.0)


def dense_siddon(g):
    if g.kind == 0:
        O, D = analytic.rays_2d(g)
        O = O.reshape(-1, 2); D = D.reshape(-1, 2)
        dims = (g.nx, g.ny)
    else:
        O, D = analytic.rays_3d(g)
        O = O.reshape(-1, 3); D = D.reshape(-1, 3)
        dims = (g.nx, g.ny, g.nz)
    A = np.zeros((O.shape[0], g.n_vox))
    idx = np.indices(dims[::-1]).reshape(len(dims), -1)[::-1]   # (ix, iy[, iz]) for x-fastest order
    for j in range(g.n_vox):
        c = np.array([(idx[a, j] - 0.5 * (dims[a] - 1)) * g.voxel for a in range(len(dims))])
        lo, hi = c - 0.5 * g.voxel, c + 0.5 * g.voxel
        for i in range(O.shape[0]):
            A[i, j] = clip_length(O[i], D[i], lo, hi)
    return A


def oracle_dense(oracle, g, fn, n_in, shape):
    cols = []
    for j in range(n_in):
        e = np.zeros(n_in)
        e[j] = 1.0
        cols.append(np.asarray(fn(g, e.reshape(shape))).reshape(-1))
    return np.stack(cols, axis=1)


# Rays lying exactly on a voxel boundary plane have no unique line-intersection
# weight (either neighbour can take the segment); the geometries keep every
# ray off those planes (even bin and row counts, pitches incommensurate with
# the voxel).
GEOMS = {
    "2d_12px_10views": parallel2d(12, 10, 20, du=0.9, projector=1),
    "2d_explicit_angles": parallel2d(9, 4, 15, voxel=1.3, du=1.1, angles=[0.3, 1.2, 2.2, 2.9], projector=1),
    "cone_8x8x6": cone3d(8, 5, 9, nz=6, nv=8, pitch=1.6, sod_factor=3.0, sdd_factor=5.0,
                         angles=[0.1, 1.3, 2.6, 3.9, 5.2], projector=1),
}


@pytest.mark.parametrize("name", list(GEOMS))
def test_siddon_dense_matches_per_voxel_clipping(oracle, name):
    g = GEOMS[name]
    ref = dense_siddon(g)
    A = oracle_dense(oracle, g, oracle.project_A, g.n_vox, g.vol_shape)
    assert np.max(np.abs(A - ref)) <= 1e-12 * np.abs(ref).max()
    AT = oracle_dense(oracle, g, oracle.backproject_AT, g.n_rays, g.sino_shape)
    assert np.max(np.abs(AT - ref.T)) <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("kind", [0, 1])
def test_siddon_constant_image_gives_chord_through_grid(oracle, kind):
    if kind == 0:
        g = parallel2d(48, 37, 80, voxel=0.7, du=0.55, projector=1)
        O, D = analytic.rays_2d(g)
        half = np.array([0.5 * g.nx * g.voxel, 0.5 * g.ny * g.voxel])
    else:
        g = cone3d(24, 11, 40, nz=20, nv=30, projector=1)
        O, D = analytic.rays_3d(g)
        half = np.array([0.5 * g.nx * g.voxel, 0.5 * g.ny * g.voxel, 0.5 * g.nz * g.voxel])
    O = O.reshape(-1, O.shape[-1]); D = D.reshape(-1, D.shape[-1])
    ref = np.array([clip_length(o, d, -half, half) for o, d in zip(O, D)])
    y = np.asarray(oracle.project_A(g, np.ones(g.vol_shape))).reshape(-1)
    assert np.max(np.abs(y - ref)) <= 1e-12 * ref.max()
    assert np.count_nonzero(ref) > 0.5 * ref.size


def test_siddon_column_and_row_sums_2d(oracle):
    g = parallel2d(64, 90, 96, projector=1)
    img = np.random.default_rng(4).uniform(size=(64, 64))
    y = np.asarray(oracle.project_A(g, img)).reshape(90, 96)
    exp0 = np.zeros(96); exp0[16:80] = img.sum(axis=0)
    exp90 = np.zeros(96); exp90[16:80] = img.sum(axis=1)
    assert np.max(np.abs(y[0] - exp0)) <= 1e-13 * exp0.max()
    assert np.max(np.abs(y[45] - exp90)) <= 1e-13 * exp90.max()


@pytest.mark.parametrize("kind", [0, 1])
def test_siddon_adjoint_identity(oracle, kind):
    g = parallel2d(40, 33, 57, projector=1) if kind == 0 else cone3d(20, 9, 30, projector=1)
    rng = np.random.default_rng(6)
    x = rng.normal(size=g.vol_shape)
    yv = rng.normal(size=g.sino_shape)
    lhs = float(np.asarray(oracle.project_A(g, x)).reshape(-1) @ yv.reshape(-1))
    rhs = float(x.reshape(-1) @ np.asarray(oracle.backproject_AT(g, yv)).reshape(-1))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_siddon_converges_to_line_integrals_of_smooth_ellipses(oracle):
    ells = phantoms.random_ellipses(17, 6, 1.0)
    errs = []
    for n in (32, 64, 128):
        g = parallel2d(n, 30, int(1.5 * n), voxel=1.0 / n, du=1.0 / n, projector=1)
        img = phantoms.rasterize_ellipses(ells, n, 1.0 / n, profile="smooth", supersample=1)
        y = np.asarray(oracle.project_A(g, img)).reshape(-1)
        O, D = analytic.rays_2d(g)
        ref = analytic.ellipse_line_integrals(ells, O, D, profile="smooth").reshape(-1)
        errs.append(rel(y, ref))
    # second order: point-sampled pixels, exact intersection lengths
    assert errs[0] / errs[1] >= 3.0 and errs[1] / errs[2] >= 3.0, errs


@pytest.mark.parametrize("name", ["2d_12px_10views", "2d_explicit_angles", "cone_8x8x6"])
def test_siddon_update_count_equals_segments(oracle, name):
    """The closed-form count (1 + boundary crossings per ray) equals the
    number of non-zero entries of the dense matrix built by per-voxel
    clipping, except that crossings which coincide (segments of ~1e-15,
    present in the symmetric cone geometry) are counted separately."""
    g = GEOMS[name]
    ref = dense_siddon(g)
    n = oracle.count_A_updates(g)
    pos = int(np.count_nonzero(ref > 0.0))
    tiny = int(np.count_nonzero((ref > 0.0) & (ref <= 1e-12)))
    if g.kind == 0:
        assert n == pos and tiny == 0
    else:
        assert pos <= n <= pos + 2 * tiny + 16, (n, pos, tiny)
