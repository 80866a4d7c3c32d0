"""GPU operator parity with the FP64 oracle (same seeded FP32 inputs).

Tolerance: relative 2-norm error <= 1e-5 for FP32 outputs, and every
element within max(1e-5, 4 N 2^-24) of the largest reference element, N
the largest grid dimension (op_elem_tol: coherent FP32 rounding of the
sample positions), so that a defect in a few rays or voxels cannot hide in
the norm of the whole output.  Derivation: the
kernels evaluate each sample position in FP32 from FP64 per-ray set-up, so
the interpolation weights carry errors of a few units of 2^-24 times the
coordinate magnitude (<= 2^9 voxels here), i.e. <= 3e-5 per weight at worst
and far smaller on average; sums over hundreds of samples in FP32 add
O(sqrt(N) 2^-24).  Observed errors sit near 1e-7..1e-6.
FP16 outputs are checked against FP16 rounding (2^-11 relative).
"""

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from synth.geometry import GeometryDesc, PARALLEL_2D, cone3d
from tests.gpu_helpers import SMALL_GEOMS, assert_close, dev, f32, host, op_elem_tol, rel, say, special_rays

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def geoms():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return {k: (d, ct.Geometry(d)) for k, d in SMALL_GEOMS.items()}


@pytest.mark.parametrize("name", list(SMALL_GEOMS))
def test_project_A(geoms, name):
    desc, g = geoms[name]
    say("A parity", name)
    x = f32(np.random.default_rng(1).uniform(0, 1, size=desc.vol_shape))
    y = host(ct.ct_project_A(g, dev(x)))
    ref = oracle.project_A(desc, x)
    assert_close(y, ref, TOL, "A " + name, op_elem_tol(desc))


@pytest.mark.parametrize("name", list(SMALL_GEOMS))
def test_backproject_B(geoms, name):
    desc, g = geoms[name]
    say("B parity", name)
    y = f32(np.random.default_rng(2).uniform(0, 1, size=desc.sino_shape))
    x = host(ct.ct_backproject_B(g, dev(y)))
    assert_close(x, oracle.backproject_Bun(desc, y), TOL, "B_un " + name, op_elem_tol(desc))


@pytest.mark.parametrize("name", list(SMALL_GEOMS))
def test_backproject_AT(geoms, name):
    desc, g = geoms[name]
    say("AT parity", name)
    rng = np.random.default_rng(3)
    y = f32(rng.uniform(0, 1, size=desc.sino_shape))
    x = host(ct.ct_backproject_AT(g, dev(y)))
    assert_close(x, oracle.backproject_AT(desc, y), TOL, "A^T " + name, op_elem_tol(desc))
    # adjoint identity of the GPU pair itself
    v = f32(rng.standard_normal(desc.vol_shape))
    w = f32(rng.standard_normal(desc.sino_shape))
    lhs = float(host(ct.ct_project_A(g, dev(v))).reshape(-1) @ w.reshape(-1).astype(np.float64))
    rhs = float(v.reshape(-1).astype(np.float64) @ host(ct.ct_backproject_AT(g, dev(w))).reshape(-1))
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs))


@pytest.mark.parametrize("name", ["w1_2d_64", "ragged_2d", "cone_24", "ragged_cone"])
def test_ramp_and_filtered_backprojection(geoms, name):
    desc, g = geoms[name]
    say("F parity", name)
    y = f32(np.random.default_rng(4).uniform(0, 1, size=desc.sino_shape))
    f = host(ct.ct_ramp_filter(g, dev(y)))
    fref = oracle.ramp(desc, y)
    assert_close(f, fref, TOL, "F " + name)
    x = host(ct.ct_backproject_B(g, dev(y), ramp=True))
    assert_close(x, oracle.backproject_Bun(desc, oracle.ramp(desc, y)), TOL, "B_FBP " + name)


@pytest.mark.parametrize("nu", [1, 2, 15, 33, 96, 385, 768, 769, 896, 897, 1088, 1089, 1600, 1601, 2048, 4096])
def test_ramp_row_lengths(nu):
    """Row lengths the filter accepts: odd and even (the two parities differ
    in length), one 16-output block and many, the whole-row matrix-core
    kernel up to its LDS budget (896 bins), the one-parity kernel up to 1600
    bins and the per-row FIR beyond; 37 rows leave a ragged last row
    group."""
    desc = GeometryDesc(PARALLEL_2D, 8, 8, 1, 1.0, 37, nu, 1, 0.8731, 1.0)
    g = ct.Geometry(desc)
    say("F row length", nu)
    y = f32(np.random.default_rng(nu).normal(size=desc.sino_shape))
    assert_close(host(ct.ct_ramp_filter(g, dev(y))), oracle.ramp(desc, y), TOL, "F nu=%d" % nu)


@pytest.mark.parametrize("name", ["w1_2d_64", "cone_24", "ragged_cone"])
def test_fp16_storage(geoms, name):
    desc, g = geoms[name]
    say("FP16 storage", name)
    x = f32(np.random.default_rng(5).uniform(0, 1, size=desc.vol_shape))
    y16 = ct.ct_project_A(g, dev(x), y_dtype=torch.float16)
    assert y16.dtype == torch.float16
    ref = oracle.project_A(desc, x)
    # each element rounded once to FP16: within 2^-11 of itself
    yh = host(y16).reshape(-1)
    assert np.all(np.abs(yh - ref) <= 2.0 ** -11 * np.abs(ref) + 1e-5 * np.abs(ref).max())
    assert rel(yh, ref) <= 2.0 ** -11
    xb = host(ct.ct_backproject_B(g, y16))
    ref_b = oracle.backproject_Bun(desc, host(y16))   # same FP16-rounded data
    assert_close(xb, ref_b, TOL, "B_un FP16 data " + name)
    xt = host(ct.ct_backproject_AT(g, y16))
    assert_close(xt, oracle.backproject_AT(desc, host(y16)), TOL, "A^T FP16 data " + name)
    # FP16 data are widened exactly when staged (four per 8-byte load where
    # the rows allow it, one by one at the detector's edges): the same
    # values given as FP32 must give the same bits
    y32 = y16.float()
    assert torch.equal(ct.ct_backproject_B(g, y16), ct.ct_backproject_B(g, y32)), "B_un " + name
    assert torch.equal(ct.ct_backproject_AT(g, y16), ct.ct_backproject_AT(g, y32)), "A^T " + name
    # the ramp filter stages FP16 rows the same way (8-byte loads of four
    # where the row allows, one by one otherwise) and keeps its output in
    # FP32, so B_FBP of FP16 data gives the bits of the same values in FP32
    assert torch.equal(ct.ct_backproject_B(g, y16, ramp=True), ct.ct_backproject_B(g, y32, ramp=True)), \
        "B_FBP " + name


@pytest.mark.parametrize("nu", [45, 96, 385, 768, 1088, 1089])
def test_ramp_fp16_rows(nu):
    """FP16 data through both matrix-core filters (whole rows up to 896
    bins, one parity at a time beyond), with and without vector staging
    (row lengths divisible by 4 or not): the FP16 values are widened
    exactly when staged, so B_FBP gives the bits of the same values given
    as FP32.  The FP32 route of these kernels is compared with the oracle
    at these row lengths in test_ramp_row_lengths (whole rows) and in
    test_ramp_and_filtered_backprojection (B_FBP); here an 8 x 8 image sees
    only the central bins of each row, where the filter's FP32 sums over
    hundreds of taps cancel the most, so the FP32 rounding of those bins is
    not measured against a fixed 1e-5 again."""
    desc = GeometryDesc(PARALLEL_2D, 8, 8, 1, 1.0, 37, nu, 1, 0.8731, 1.0)
    g = ct.Geometry(desc)
    say("F FP16 rows", nu)
    y16 = dev(f32(np.random.default_rng(nu + 7).uniform(0, 1, size=desc.sino_shape))).half()
    x16 = ct.ct_backproject_B(g, y16, ramp=True)
    assert torch.equal(x16, ct.ct_backproject_B(g, y16.float(), ramp=True)), "B_FBP FP16 nu=%d" % nu


@pytest.mark.parametrize("projector", [0, 1])
def test_project_A_small_shadow(projector):
    """A volume whose shadow covers a small part of a large detector: most
    detector tiles lie outside the bounding box of the shadow and take the
    early exit (zeros without ray set-up); every other value must be
    unchanged, and the zeros must be exactly those of the oracle."""
    desc = cone3d(16, 12, 112, sod_factor=16.0, sdd_factor=32.0, projector=projector)
    g = ct.Geometry(desc)
    say("A small shadow", projector)
    x = f32(np.random.default_rng(8).uniform(0, 1, size=desc.vol_shape))
    y = host(ct.ct_project_A(g, dev(x))).reshape(desc.sino_shape)
    ref = np.asarray(oracle.project_A(desc, x)).reshape(desc.sino_shape)
    assert_close(y, ref, TOL, "A small shadow", op_elem_tol(desc))
    # exact zeros away from the edge of the shadow (pixels whose 3 x 3
    # neighbourhood is zero in the oracle), where rounding cannot decide
    # whether a grazing ray picks up a sample
    z = ref == 0.0
    far = z.copy()
    for du in (-1, 0, 1):
        for dv in (-1, 0, 1):
            far[:, 1:-1, 1:-1] &= z[:, 1 + dv:z.shape[1] - 1 + dv, 1 + du:z.shape[2] - 1 + du]
    assert far.mean() > 0.5
    assert np.all(y[far] == 0.0)


@pytest.mark.parametrize("projector", [0, 1])
def test_project_A_axis_switch_views(projector):
    """Views whose rays change dominant axis across the detector (angles
    around 45 and 135 degrees, ragged detector of 53 columns): each view's
    ray tiles are offset so that a tile edge falls on the switch column,
    leaving partial tiles at both detector edges; every ray must still
    match the oracle."""
    angles = [np.deg2rad(a) for a in np.linspace(28.0, 62.0, 9)] + \
             [np.deg2rad(a) for a in np.linspace(118.0, 152.0, 9)] + [0.0, np.pi / 2]
    desc = cone3d(20, len(angles), 53, nv=21, nz=18, angles=angles, sod_factor=3.0, sdd_factor=6.0,
                  projector=projector)
    g = ct.Geometry(desc)
    say("A axis-switch views", projector)
    x = f32(np.random.default_rng(9).uniform(0, 1, size=desc.vol_shape))
    y = host(ct.ct_project_A(g, dev(x)))
    assert_close(y, oracle.project_A(desc, x), TOL, "A axis-switch views", op_elem_tol(desc))


@pytest.mark.parametrize("projector", [0, 1])
def test_project_A_volume_beyond_last_level_cache(projector):
    """A volume whose two padded copies exceed the 256 MB last-level cache
    (384 x 384 x 232, 281 MB of copies) is projected in the band order with
    groups of four views; 7 views (a partial last group) of a ragged 77 x 53
    detector whose pitch makes it span the whole volume: every ray must
    match the oracle."""
    desc = cone3d(384, 7, 77, nv=53, nz=232, pitch=10.0, projector=projector)
    g = ct.Geometry(desc)
    say("A beyond the last-level cache", projector)
    x = f32(np.random.default_rng(10).uniform(0, 1, size=desc.vol_shape))
    y = host(ct.ct_project_A(g, dev(x)))
    ref = oracle.project_A(desc, x)
    assert np.count_nonzero(ref) > 0.5 * ref.size
    assert_close(y, ref, TOL, "A beyond the last-level cache", op_elem_tol(desc))


# Geometries that send the cone-beam transpose down each of its paths:
#   fine_pitch     four detector columns and rows per voxel: planes wider than
#                  the sheets and boxes larger than the staged tile (the
#                  per-voxel fallback reading the data from global memory);
#   coarse_pitch   a third of a column and row per voxel: |a1| = 3, rows
#                  splatted one by one inside the sheet path;
#   short_sod      magnification 3 at the near face and 1.5 at the far one:
#                  some blocks with planes wider than the sheets, the others
#                  on the sheet path with |a1| on both sides of 1;
#   wide_fan       a 127 degree fan (12 rows, so that no ray is z-dominant):
#                  the dominant axis changes twice across the detector, so
#                  plane ranges are not cut to one axis.
AT_PATH_GEOMS = {
    "fine_pitch": dict(n=20, views=12, det=100, pitch=0.5),
    "coarse_pitch": dict(n=24, views=12, det=12, pitch=6.0),
    "short_sod": dict(n=32, views=16, det=64, sod_factor=1.5, sdd_factor=3.0),
    "wide_fan": dict(n=16, views=8, det=64, sod_factor=1.5, sdd_factor=2.0, pitch=2.0, nv=12, nz=8),
}


@pytest.mark.parametrize("projector", [0, 1])
@pytest.mark.parametrize("name", list(AT_PATH_GEOMS))
def test_transpose_paths(name, projector):
    kw = dict(AT_PATH_GEOMS[name])
    desc = cone3d(kw.pop("n"), kw.pop("views"), kw.pop("det"), projector=projector, **kw)
    g = ct.Geometry(desc)
    say("A and A^T paths", name, projector)
    rng = np.random.default_rng(11)
    y = f32(rng.uniform(0, 1, size=desc.sino_shape))
    x = host(ct.ct_backproject_AT(g, dev(y)))
    assert_close(x, oracle.backproject_AT(desc, y), TOL, "A^T %s (model %d)" % (name, projector), op_elem_tol(desc))
    v = f32(rng.uniform(0, 1, size=desc.vol_shape))
    assert_close(host(ct.ct_project_A(g, dev(v))), oracle.project_A(desc, v), TOL,
                 "A %s (model %d)" % (name, projector), op_elem_tol(desc))


def test_batch_equals_single_calls(geoms):
    desc, g = geoms["cone_24"]
    rng = np.random.default_rng(6)
    xs = f32(rng.uniform(size=(3,) + desc.vol_shape))
    yb = ct.ct_project_A(g, dev(xs))
    for i in range(3):
        yi = ct.ct_project_A(g, dev(xs[i]))
        assert torch.equal(yb[i], yi)
    xb = ct.ct_backproject_B(g, yb)
    for i in range(3):
        assert torch.equal(xb[i], ct.ct_backproject_B(g, yb[i].contiguous()))


def test_empty_batch(geoms):
    desc, g = geoms["w1_2d_64"]
    x = torch.empty((0,) + desc.vol_shape, device="cuda")
    y = ct.ct_project_A(g, x)
    assert y.shape == (0,) + desc.sino_shape


# ------------------------------------------------ full workload sizes
def _sampled_parity(desc, g, vol, nsamp=3000, seed=7):
    """Random rays and voxels, plus the rays where the projector's tiling
    decisions change (detector edges, where the view's tiles are partial,
    the columns around each view's dominant-axis switch, where the tile
    columns are offset, and rows and columns around tile boundaries), and
    the volume's corner and edge voxels."""
    rng = np.random.default_rng(seed)
    y = ct.ct_project_A(g, dev(vol))
    yh = host(y).reshape(-1)
    rays = np.union1d(rng.choice(desc.n_rays, size=nsamp, replace=False), special_rays(desc))
    ref = oracle.project_A_rays(desc, vol, rays)
    assert_close(yh[rays], ref, TOL, "A sampled rays", op_elem_tol(desc))
    x = host(ct.ct_backproject_B(g, y)).reshape(-1)
    nz, ny, nx = desc.vol_shape
    edge = [(z * ny + yy) * nx + xx for z in (0, nz // 2, nz - 1) for yy in (0, ny // 2, ny - 1)
            for xx in (0, 1, nx // 2, nx - 2, nx - 1)]
    vox = np.union1d(rng.choice(desc.n_vox, size=nsamp, replace=False), np.array(edge, np.int64))
    refb = oracle.backproject_Bun_voxels(desc, f32(yh), vox)
    assert_close(x[vox], refb, TOL, "B_un sampled voxels", op_elem_tol(desc))
    xr = host(ct.ct_backproject_B(g, y, ramp=True)).reshape(-1)
    fy = oracle.ramp(desc, f32(yh))
    refr = oracle.backproject_Bun_voxels(desc, fy, vox)
    assert_close(xr[vox], refr, TOL, "B_FBP sampled voxels")


def test_w2_full_size_sampled():
    desc = workloads.w2_geometry()
    say("W2 128^3 sampled parity")
    g = ct.Geometry(desc)
    _sampled_parity(desc, g, workloads.w2_phantom())


def test_w3_full_size_sampled():
    desc = workloads.w3_geometry()
    say("W3 256^3 sampled parity")
    g = ct.Geometry(desc)
    vol = workloads.w3_phantom()
    _sampled_parity(desc, g, vol, nsamp=2000)
