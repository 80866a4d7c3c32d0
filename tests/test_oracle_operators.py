"""Pins of the FP64 oracle operators against closed forms, invariants and
special cases that do not reuse the oracle's own formulas.

A   Joseph projector      column/row sums at 0 and 90 deg, chord lengths of a
                          constant image, second-order convergence to the
                          exact line integrals of smooth ellipses/ellipsoids,
                          90-degree rotation covariance, update counts.
A^T transpose             adjoint identity.
B   voxel-driven B_un     single-view special case, back-projection of a
                          Gaussian's exact sinogram (Bessel closed form),
                          exact bilinear reproduction of a linear detector
                          function with a projection computed by a 3x3 solve,
                          A/B geometric consistency, unmatched by design.
F   Ram-Lak filter        exact ramp-filtered Gaussian (Dawson closed form),
                          symmetry.
"""

import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import i0e

from synth.geometry import GeometryDesc, parallel2d, cone3d, PARALLEL_2D, CONE_3D
from synth import phantoms
from tests import analytic


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


# ------------------------------------------------------------------ A, 2D
def test_joseph2d_column_and_row_sums(oracle):
    """At 0 deg the rays run along +y through pixel columns (f_x integer), so
    A x is the column sum; at 90 deg it is the row sum (unit pixel, bin)."""
    g = parallel2d(64, 90, 96)
    rng = np.random.default_rng(1)
    img = rng.uniform(0, 1, size=(64, 64))
    y = oracle.project_A(g, img).reshape(90, 96)
    col = img.sum(axis=0)          # over iy for each ix
    row = img.sum(axis=1)          # over ix for each iy
    exp0 = np.zeros(96); exp0[16:80] = col
    exp90 = np.zeros(96); exp90[16:80] = row
    assert np.max(np.abs(y[0] - exp0)) <= 1e-14 * np.abs(exp0).max()
    assert np.max(np.abs(y[45] - exp90)) <= 1e-14 * np.abs(exp90).max()


def _box_chords_2d(g, O, D):
    """Chord length of each ray between the two faces of the image box
    perpendicular to its dominant axis, and whether the ray stays at least
    half a pixel inside the other pair of faces between them."""
    half = 0.5 * g.nx * g.voxel
    inner = 0.5 * (g.nx - 1) * g.voxel
    a = np.where(np.abs(D[..., 0]) >= np.abs(D[..., 1]), 0, 1)
    chords = np.zeros(O.shape[:-1])
    ok = np.zeros(O.shape[:-1], bool)
    for idx in np.ndindex(O.shape[:-1]):
        ax = a[idx]; ot = 1 - ax
        o, d = O[idx], D[idx]
        t1 = (-half - o[ax]) / d[ax]
        t2 = (half - o[ax]) / d[ax]
        p1, p2 = o + t1 * d, o + t2 * d
        chords[idx] = np.linalg.norm(p2 - p1)
        ok[idx] = abs(p1[ot]) <= inner - 1e-9 and abs(p2[ot]) <= inner - 1e-9
    return chords, ok, a


def test_joseph2d_constant_image_chord_length(oracle):
    g = parallel2d(32, 30, 48, angles=[(p + 0.31) * math.pi / 30 for p in range(30)])
    y = oracle.project_A(g, np.ones((32, 32))).reshape(30, 48)
    O, D = analytic.rays_2d(g)
    chords, ok, _ = _box_chords_2d(g, O, D)
    assert ok.sum() > 200
    # Joseph samples the N voxel-centre planes; its support reaches half a voxel
    # beyond them, i.e. to the faces, so the chord is N*vox*|r|/|r_a|.
    np.testing.assert_allclose(y[ok], chords[ok], rtol=1e-13)


def test_joseph3d_constant_volume_chord_length(oracle):
    g = cone3d(16, 12, 24)
    y = oracle.project_A(g, np.ones((16, 16, 16))).reshape(12, 24, 24)
    O, D = analytic.rays_3d(g)
    half = 8.0; inner = 7.5
    checked = 0
    for idx in np.ndindex(O.shape[:-1]):
        o, d = O[idx], D[idx]
        ax = int(np.argmax(np.abs(d)))
        t1, t2 = (-half - o[ax]) / d[ax], (half - o[ax]) / d[ax]
        p1, p2 = o + t1 * d, o + t2 * d
        others = [k for k in range(3) if k != ax]
        if all(abs(p1[k]) <= inner - 1e-9 and abs(p2[k]) <= inner - 1e-9 for k in others):
            assert abs(y[idx] - np.linalg.norm(p2 - p1)) <= 1e-12 * np.linalg.norm(p2 - p1)
            checked += 1
    assert checked > 100


def _smooth_2d_error(oracle, n):
    fov = 64.0
    vox = fov / n
    ells = phantoms.random_ellipses(7, 6, fov)
    img = phantoms.rasterize_ellipses(ells, n, vox, profile="smooth")
    angles = [(p + 0.37) * math.pi / 24 for p in range(24)]
    g = GeometryDesc(PARALLEL_2D, n, n, 1, vox, 24, 80, 1, 1.2, 1.0, angles=tuple(angles))
    y = oracle.project_A(g, img)
    O, D = analytic.rays_2d(g)
    exact = analytic.ellipse_line_integrals(ells, O, D, "smooth").reshape(-1)
    return rel(y, exact)


def test_joseph2d_second_order_convergence_smooth_ellipses(oracle):
    e = [_smooth_2d_error(oracle, n) for n in (64, 128, 256)]
    assert e[0] / e[1] >= 3.0 and e[1] / e[2] >= 3.0, e
    assert e[2] < 1e-3


def _smooth_3d_error(oracle, n):
    fov = 64.0
    vox = fov / n
    ells = phantoms.random_ellipsoids(11, 5, fov)
    vol = phantoms.rasterize_ellipsoids(ells, n, vox, profile="smooth")
    angles = tuple((p + 0.23) * 2 * math.pi / 8 for p in range(8))
    g = GeometryDesc(CONE_3D, n, n, n, vox, 8, 40, 40, 3.2, 3.2, 256.0, 512.0, angles)
    y = oracle.project_A(g, vol)
    O, D = analytic.rays_3d(g)
    exact = analytic.ellipsoid_line_integrals(ells, O, D, "smooth").reshape(-1)
    return rel(y, exact)


@pytest.mark.slow
def test_joseph3d_second_order_convergence_smooth_ellipsoids(oracle):
    e = [_smooth_3d_error(oracle, n) for n in (32, 64, 128)]
    assert e[0] / e[1] >= 3.0 and e[1] / e[2] >= 3.0, e


def _uniform_3d_error(oracle, n):
    fov = 64.0
    vox = fov / n
    ells = phantoms.random_ellipsoids(13, 6, fov)
    vol = phantoms.rasterize_ellipsoids(ells, n, vox)
    angles = tuple((p + 0.41) * 2 * math.pi / 6 for p in range(6))
    g = GeometryDesc(CONE_3D, n, n, n, vox, 6, 48, 48, 2.7, 2.7, 256.0, 512.0, angles)
    y = oracle.project_A(g, vol)
    O, D = analytic.rays_3d(g)
    exact = analytic.ellipsoid_line_integrals(ells, O, D, "uniform").reshape(-1)
    return rel(y, exact)


def test_joseph3d_uniform_ellipsoids_error_decreases(oracle):
    """Uniform (discontinuous) ellipsoids: the error is limited by the
    point-sampled edges, so only a decrease with resolution is asserted."""
    e = [_uniform_3d_error(oracle, n) for n in (32, 64, 128)]
    assert e[0] > e[1] > e[2], e


def test_joseph2d_rotation_covariance(oracle):
    """Rotating the image by +90 deg shifts the sinogram by P/2 views, with
    the bin order reversed for the views that wrap past 180 deg."""
    g = parallel2d(40, 90, 60)
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, size=(40, 40))
    # +90 deg about the centre: new(X, Y) = old(Y, -X)
    # -> new[iy][ix] = old[N-1-ix][iy]
    rot = np.empty_like(img)
    for iy in range(40):
        for ix in range(40):
            rot[iy, ix] = img[40 - 1 - ix, iy]
    y = oracle.project_A(g, img).reshape(90, 60)
    yr = oracle.project_A(g, rot).reshape(90, 60)
    exp = np.empty_like(y)
    exp[45:] = y[:45]
    exp[:45] = y[45:, ::-1]
    assert np.max(np.abs(yr - exp)) <= 1e-12 * np.abs(y).max()


def test_update_counts_special_cases(oracle):
    """At 0 and 90 deg exactly 64 bins see the 64x64 image, 64 planes each."""
    g = parallel2d(64, 2, 96)          # views 0 and 90 deg
    assert oracle.count_A_updates(g) == 2 * 64 * 64
    # 4x4 central detector pixels of a 16^3 cone geometry: every ray stays
    # within 1.7 voxels of the axis, so all 16 planes count for each ray
    g3 = cone3d(16, 1, 4, angles=[0.0])
    assert oracle.count_A_updates(g3) == 16 * 16


# ---------------------------------------------------------------- A^T
@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_adjoint_identity(oracle, kind):
    if kind == "2d":
        g = parallel2d(48, 45, 70)
    else:
        g = cone3d(24, 20, 36)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(g.n_vox)
    y = rng.standard_normal(g.n_rays)
    lhs = float(oracle.project_A(g, x) @ y)
    rhs = float(x @ oracle.backproject_AT(g, y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------------------ B_un
def test_bun2d_single_view_theta0(oracle):
    g = parallel2d(64, 1, 96)         # single view at 0 deg
    rng = np.random.default_rng(2)
    y = rng.uniform(size=96)
    x = oracle.backproject_Bun(g, y).reshape(64, 64)
    exp = np.broadcast_to(y[16:80][None, :], (64, 64))
    assert np.array_equal(x, exp)
    xt = oracle.backproject_AT(g, y).reshape(64, 64)
    np.testing.assert_allclose(xt, exp, rtol=1e-15, atol=0)


def _bun_gaussian_error(oracle, h):
    """Exact parallel projection of exp(-r^2/(2 s^2)) is s sqrt(2 pi)
    exp(-t^2/(2 s^2)) in every view; its back-projection over [0, pi) is
    pi s sqrt(2 pi) exp(-r^2/(4 s^2)) I0(r^2/(4 s^2))."""
    sigma = 6.0
    n = int(round(48 / h))
    P = 180
    nu = int(round(72 / h))
    g = parallel2d(n, P, nu, voxel=h, du=h)
    t = (np.arange(nu) - 0.5 * (nu - 1)) * h
    sino = np.tile(sigma * math.sqrt(2 * math.pi) * np.exp(-t ** 2 / (2 * sigma ** 2)), P)
    x = oracle.backproject_Bun(g, sino).reshape(n, n)
    c = (np.arange(n) - 0.5 * (n - 1)) * h
    r2 = c[None, :] ** 2 + c[:, None] ** 2
    exact = math.pi * sigma * math.sqrt(2 * math.pi) * i0e(r2 / (4 * sigma ** 2))
    # weight vox^2/du per view approximates (pi/P) d(theta) * (vox^2/du) ...
    scaled = x * (math.pi * g.du) / (P * g.voxel ** 2)
    mask = r2 < 20.0 ** 2
    return rel(scaled[mask], exact[mask])


def test_bun2d_gaussian_bessel_closed_form(oracle):
    e = [_bun_gaussian_error(oracle, h) for h in (1.0, 0.5, 0.25)]
    assert e[0] < 5e-3, e
    assert e[0] / e[1] >= 3.0 and e[1] / e[2] >= 3.0, e


def _project_point_cone(g, theta, p):
    """(t, u, v) with source + t (p - source) = centre + u e_u + v e_v."""
    src, cen, eu, ev = analytic.cone_frame(g, theta)
    Mtx = np.stack([p - src, -eu, -ev], axis=1)
    return np.linalg.solve(Mtx, cen - src)


def test_bun3d_reproduces_linear_detector_function(oracle):
    theta = 0.61
    g = cone3d(20, 1, 40, angles=[theta])
    a, b, c = 0.37, -0.21, 1.5
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du
    v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.dv
    sino = (a * u[None, :] + b * v[:, None] + c).reshape(-1)
    x = oracle.backproject_Bun(g, sino).reshape(20, 20, 20)
    rng = np.random.default_rng(9)
    checked = 0
    for _ in range(200):
        iz, iy, ix = rng.integers(0, 20, size=3)
        pt = (np.array([ix, iy, iz]) - 9.5) * g.voxel
        t, uu, vv = _project_point_cone(g, theta, pt)
        if abs(uu) < u[-1] - g.du and abs(vv) < v[-1] - g.dv:
            exp = g.voxel ** 3 * t * t / (g.du * g.dv) * (a * uu + b * vv + c)
            assert abs(x[iz, iy, ix] - exp) <= 1e-12 * abs(exp)
            checked += 1
    assert checked > 150


def test_projector_backprojector_geometric_consistency(oracle):
    """The detector centroid of A e_j equals where B_un projects voxel j.
    A fine detector (1/8 voxel at the isocentre) samples the footprint well
    enough for its centroid to resolve 0.05 pixel."""
    g = cone3d(16, 6, 200, pitch=0.25)
    th = analytic.angles_of(g)
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du
    v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.dv
    rng = np.random.default_rng(4)
    for _ in range(6):
        iz, iy, ix = rng.integers(3, 13, size=3)
        e = np.zeros((16, 16, 16)); e[iz, iy, ix] = 1.0
        y = oracle.project_A(g, e).reshape(g.n_views, g.nv, g.nu)
        pt = (np.array([ix, iy, iz]) - 7.5) * g.voxel
        for p in range(g.n_views):
            w = y[p]
            cu = (w.sum(0) * u).sum() / w.sum()
            cv = (w.sum(1) * v).sum() / w.sum()
            _, uu, vv = _project_point_cone(g, th[p], pt)
            assert abs(cu - uu) <= 0.05 * g.du and abs(cv - vv) <= 0.05 * g.dv


def test_bun_is_unmatched_but_close_in_scale(oracle):
    g = parallel2d(16, 24, 24)
    n, m = 256, 24 * 24
    AT = np.stack([oracle.backproject_AT(g, np.eye(m)[i]) for i in range(m)], axis=1)
    B = np.stack([oracle.backproject_Bun(g, np.eye(m)[i]) for i in range(m)], axis=1)
    diff = np.linalg.norm(B - AT) / np.linalg.norm(AT)
    assert diff >= 1e-3
    ones = np.ones(m)
    ratio = (B @ ones).reshape(16, 16)[4:12, 4:12] / (AT @ ones).reshape(16, 16)[4:12, 4:12]
    assert np.all(np.abs(ratio - 1.0) < 0.1)


# ------------------------------------------------------------------ F
def test_ramp_closed_form_identity():
    """Check the Dawson closed form of the ramp-filtered Gaussian by quadrature."""
    sigma = 2.5
    for x0 in (0.0, 1.3, 4.0, 9.0):
        a = 2 * math.pi ** 2 * sigma ** 2
        f = lambda k: k * math.exp(-a * k * k) * math.cos(2 * math.pi * x0 * k)
        val, _ = integrate.quad(f, 0, 10.0 / sigma, limit=400)
        exp = 2 * sigma * math.sqrt(2 * math.pi) * val
        assert abs(analytic.ramp_filtered_gaussian(x0, sigma) - exp) < 1e-10


@pytest.mark.parametrize("du", [1.0, 0.7])
def test_ramp_matches_continuous_ramp_of_gaussian(oracle, du):
    nu = 256
    sigma = 4.0 * du
    g = parallel2d(8, 3, nu, du=du)
    s = (np.arange(nu) - 0.5 * (nu - 1)) * du
    row = np.exp(-s ** 2 / (2 * sigma ** 2))
    out = oracle.ramp(g, np.tile(row, 3)).reshape(3, nu)
    exact = analytic.ramp_filtered_gaussian(s, sigma)
    for p in range(3):
        assert np.max(np.abs(out[p] - exact)) <= 1e-9 * np.abs(exact).max()


def test_ramp_is_symmetric(oracle):
    g = parallel2d(8, 4, 50)
    rng = np.random.default_rng(8)
    p, q = rng.standard_normal(200), rng.standard_normal(200)
    lhs = float(oracle.ramp(g, p) @ q)
    rhs = float(p @ oracle.ramp(g, q))
    assert abs(lhs - rhs) <= 1e-14 * np.abs(p).sum() * np.abs(q).sum()


# ------------------------------------------------------------------ FBP / FDK
def test_fbp2d_reconstructs_disk_and_converges(oracle):
    """Filtered back-projection of the exact sinogram of a uniform disk of
    density 1: interior values tend to 1 as the sampling is refined."""
    disk = [dict(cx=0.07, cy=-0.05, a=0.3, b=0.3, phi=0.0, rho=1.0)]
    errs = []
    for n in (64, 128, 256):
        g = parallel2d(n, 2 * n, int(1.5 * n), voxel=1.0 / n, du=1.0 / n)
        O, D = analytic.rays_2d(g)
        y = analytic.ellipse_line_integrals(disk, O, D)
        x = np.asarray(oracle.fbp(g, y)).reshape(n, n)
        c = (np.arange(n) - 0.5 * (n - 1)) / n
        X, Y = np.meshgrid(c, c)
        inside = (X - 0.07) ** 2 + (Y + 0.05) ** 2 < (0.3 - 6.0 / n) ** 2
        outside = (X - 0.07) ** 2 + (Y + 0.05) ** 2 > (0.3 + 6.0 / n) ** 2
        errs.append(float(np.sqrt(np.mean((x[inside] - 1.0) ** 2))))
        assert abs(float(np.mean(x[outside & (X ** 2 + Y ** 2 < 0.2)]))) < 0.02
    assert errs[2] < errs[1] < errs[0] and errs[2] < 0.01, errs


def test_fdk_reconstructs_ball_midplane(oracle):
    """FDK of the exact cone-beam projections of a centred ball of density
    1: close to 1 in the interior of the mid-plane, where the circular orbit
    samples the Radon space completely (a missing scale factor, weight or
    filter pitch would show as a percent-level or larger offset)."""
    errs, centres = [], []
    for n in (24, 48):
        g = cone3d(n, 4 * n, int(1.5 * n), voxel=1.0 / n)
        ball = [dict(centre=np.zeros(3), semi=np.array([0.3, 0.3, 0.3]), R=np.eye(3), rho=1.0)]
        O, D = analytic.rays_3d(g)
        y = analytic.ellipsoid_line_integrals(ball, O, D)
        x = np.asarray(oracle.fbp(g, y)).reshape(n, n, n)
        c = (np.arange(n) - 0.5 * (n - 1)) / n
        X, Y = np.meshgrid(c, c)
        mid = 0.5 * (x[n // 2 - 1] + x[n // 2])
        zc = 0.5 / n
        inside = X ** 2 + Y ** 2 + zc ** 2 < (0.3 - 4.0 / n) ** 2
        errs.append(float(np.sqrt(np.mean((mid[inside] - 1.0) ** 2))))
        centres.append(float(mid[n // 2 - 1:n // 2 + 1, n // 2 - 1:n // 2 + 1].mean()))
    assert max(errs) < 0.02, errs
    assert all(abs(c - 1.0) < 0.01 for c in centres), centres


# ------------------------------------------- sampled evaluation of A, B_un
# The full-size GPU tests and the benchmark check the GPU against the
# oracle's sampled evaluations (selected rays of A, selected voxels of
# B_un), so these must be the same numbers as the full operators pinned
# above: bit for bit, at random indices and at the first and last ray or
# voxel, for both geometries and both forward models.
_SAMPLED_GEOMS = {
    "2d": parallel2d(37, 45, 53),
    "2d_siddon": parallel2d(29, 36, 41, projector=1),
    "cone": cone3d(14, 9, 21, nz=11, nv=17),
    "cone_siddon": cone3d(12, 7, 19, projector=1),
}


@pytest.mark.parametrize("name", list(_SAMPLED_GEOMS))
def test_sampled_rays_equal_full_projection(oracle, name):
    g = _SAMPLED_GEOMS[name]
    rng = np.random.default_rng(31)
    x = rng.uniform(0.0, 1.0, size=g.vol_shape)
    full = oracle.project_A(g, x)
    ids = np.concatenate([[0, g.n_rays - 1], rng.choice(g.n_rays, size=200, replace=False),
                          [g.n_rays // 2, 0]])   # repeats are allowed
    part = oracle.project_A_rays(g, x, ids)
    assert np.count_nonzero(full[ids]) > 0.3 * ids.size
    assert np.array_equal(part, full[ids])


@pytest.mark.parametrize("name", ["2d", "cone"])
def test_sampled_voxels_equal_full_backprojection(oracle, name):
    g = _SAMPLED_GEOMS[name]
    rng = np.random.default_rng(32)
    y = rng.uniform(-1.0, 1.0, size=g.sino_shape)
    full = oracle.backproject_Bun(g, y)
    ids = np.concatenate([[0, g.n_vox - 1], rng.choice(g.n_vox, size=200, replace=False), [g.n_vox // 3]])
    part = oracle.backproject_Bun_voxels(g, y, ids)
    assert np.count_nonzero(full[ids]) > 0.9 * ids.size
    assert np.array_equal(part, full[ids])


def test_sampled_rays_cone_workload_proportions(oracle):
    """The cone-beam workloads' proportions (detector 1.5 N, SOD = 4 N,
    SDD = 8 N) at 32^3 and 18 views, on a random volume and on its own
    projection: sampled rays and voxels, plus the first and last, equal the
    full operators."""
    from synth import workloads
    g = workloads.w2_geometry(32, 18)
    rng = np.random.default_rng(33)
    x = rng.uniform(0.0, 1.0, size=g.vol_shape)
    full = oracle.project_A(g, x)
    ids = np.concatenate([[0, g.n_rays - 1], rng.choice(g.n_rays, size=500, replace=False)])
    assert np.array_equal(oracle.project_A_rays(g, x, ids), full[ids])
    fb = oracle.backproject_Bun(g, full)
    vids = np.concatenate([[0, g.n_vox - 1], rng.choice(g.n_vox, size=500, replace=False)])
    assert np.array_equal(oracle.backproject_Bun_voxels(g, full, vids), fb[vids])
