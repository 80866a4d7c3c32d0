"""Shared helpers for the GPU parity tests (inputs are seeded; the oracle
sees the exact FP64 upcast of the FP32 arrays the GPU receives)."""

import sys

import numpy as np
import torch

from synth.geometry import GeometryDesc, parallel2d, cone3d, PARALLEL_2D, CONE_3D


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def dev(a) -> torch.Tensor:
    return torch.from_numpy(f32(a)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def rel(a, b) -> float:
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def elem_err(a, b):
    """Largest element-wise distance relative to the largest reference
    element: max_i |a_i - b_i| / max_i |b_i|, and the index where it
    occurs.  Unlike the 2-norm distance, a defect confined to a few
    elements is not diluted by the size of the whole vector."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    if a.size == 0:
        return 0.0, -1
    d = np.abs(a - b)
    i = int(np.argmax(d))
    nb = float(np.max(np.abs(b)))
    return float(d[i] / (nb if nb > 0 else 1.0)), i


def op_elem_tol(desc, tol=1e-5):
    """Per-element bound for one FP32 operator application, relative to the
    largest element of the operator applied to |input|: max(tol, 4 N u),
    u = 2^-24, N the largest grid or detector dimension.  Sample positions
    are computed in FP32 from coordinates of magnitude up to about N cells,
    so every position of a ray (or voxel) can carry the same rounding of
    about 2 N u cells; coherent over the L samples of a ray, that moves the
    ray by up to 2 N u L times the largest difference of neighbouring input
    values, i.e. up to about 4 N u of the largest output for inputs in
    [0, 1] (largest over mean 2).  A wrong sample or tap moves its element
    by about 1 / L of a typical element (>= 2e-3 here), far beyond it."""
    n = max(desc.nx, desc.ny, desc.nz, desc.nu, desc.nv)
    return max(tol, 4.0 * n * 2.0 ** -24)


def assert_close(a, b, tol, what="", elem_tol=None, scale=None):
    """Both bounds at once: the relative 2-norm distance <= tol and every
    element within elem_tol (default tol) times `scale` (default the largest
    reference element; for an operator applied to signed input, the largest
    element of the operator applied to |input|, which removes the
    cancellation from the normalisation).  The message names the worst
    element."""
    e2 = rel(a, b)
    ei, i = elem_err(a, b)
    if scale is not None and i >= 0:
        nb = float(np.max(np.abs(np.asarray(b, np.float64))))
        ei = ei * nb / scale if scale > 0 else ei
    et = tol if elem_tol is None else elem_tol
    a1 = np.asarray(a, np.float64).reshape(-1)
    b1 = np.asarray(b, np.float64).reshape(-1)
    msg = "%s: rel 2-norm %.3e (tol %.1e), worst element %d: %.9g vs %.9g, %.3e of max|ref| (tol %.1e)" % (
        what, e2, tol, i, a1[i] if i >= 0 else 0.0, b1[i] if i >= 0 else 0.0, ei, et)
    say(msg)
    assert e2 <= tol and ei <= et, msg
    return e2, ei


def assert_hist_close(a, b, tol, what=""):
    """Residual histories: every entry within tol of the reference entry,
    relative to that entry (late, small residuals are not hidden behind the
    first one), plus 1e-12 of the first entry for residuals that are zero up
    to rounding (after a breakdown)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    floor = 1e-12 * abs(b[0]) if b.size else 0.0
    r = np.maximum(np.abs(a - b) - floor, 0.0) / np.maximum(np.abs(b), 1e-300)
    k = int(np.argmax(r))
    msg = "%s: residual history worst entry k=%d: %.9g vs %.9g (rel %.3e, tol %.1e)" % (what, k, a[k], b[k], r[k], tol)
    say(msg)
    assert r[k] <= tol, msg
    return float(r[k])


# small geometries spanning several tiles with ragged tails
SMALL_GEOMS = {
    "w1_2d_64": parallel2d(64, 90, 96),
    "ragged_2d": GeometryDesc(PARALLEL_2D, 37, 29, 1, 0.9, 50, 61, 1, 1.1, 1.0),
    "explicit_angles_2d": parallel2d(40, 33, 70, angles=[0.1 + 0.093 * p for p in range(33)]),
    "cone_24": cone3d(24, 20, 36),
    "ragged_cone": GeometryDesc(CONE_3D, 33, 30, 17, 1.0, 13, 45, 29, 1.7, 2.3, 140.0, 290.0),
    "cone_45deg_views": cone3d(20, 8, 30),   # views at multiples of 45 deg
    # P divisible by 4: views at exactly 45 and 135 deg, where the dominant
    # axis is decided by the integer tie rule (x-major iff P <= 4p <= 3P)
    "exact45_2d": parallel2d(64, 180, 96),
}


def special_rays(desc, views=None, rows=None):
    """Ray indices where tiling decisions of a cone-beam projector change:
    the detector's first and last columns and rows, the columns on both
    sides of each view's dominant-axis switch (where the in-plane direction
    has |r_x| = |r_y|), and row and column indices around multiples of 16.
    Computed from the geometry's definition in FP64 on the host."""
    P, nv, nu = desc.sino_shape
    if views is None:
        views = sorted(set([0, P - 1, P // 8, P // 4, (3 * P) // 8, P // 2] + list(range(0, P, max(1, P // 24)))))
    if rows is None:
        rows = sorted(set(r for r in [0, 1, 15, 16, 17, nv // 2, nv - 17, nv - 16, nv - 2, nv - 1] if 0 <= r < nv))
    angles = np.asarray(desc.angles, np.float64) if desc.angles is not None else \
        np.array([(2.0 * np.pi * p) / P for p in range(P)])
    u = (np.arange(nu) - 0.5 * (nu - 1)) * desc.du

    def switches(p):
        c, s = np.cos(angles[p]), np.sin(angles[p])
        ax = np.abs(-desc.sdd * c - u * s) >= np.abs(-desc.sdd * s + u * c)
        return np.nonzero(ax[1:] != ax[:-1])[0]

    # add up to eight views whose switch column lies inside the detector
    with_switch = [p for p in range(P) if len(switches(p)) > 0]
    views = sorted(set(views) | set(with_switch[::max(1, len(with_switch) // 8)]))
    ids = set()
    for p in views:
        c, s = np.cos(angles[p]), np.sin(angles[p])
        rx = -desc.sdd * c - u * s
        ry = -desc.sdd * s + u * c
        ax = np.abs(rx) >= np.abs(ry)
        cols = {0, 1, nu - 2, nu - 1, 15, 16, nu - 17, nu - 16}
        for a in np.nonzero(ax[1:] != ax[:-1])[0]:
            cols.update({a - 1, a, a + 1, a + 2})
        for a in cols:
            if 0 <= a < nu:
                for r in rows:
                    ids.add((p * nv + r) * nu + a)
    return np.array(sorted(ids), dtype=np.int64)


def fp32_envelope(desc, b, K, B="un", solver="ba", draws=3, seed=0, basis="f64"):
    """The iterate part of fp32_envelopes (see there)."""
    return fp32_envelopes(desc, b, K, B, solver, draws, seed, basis)[0]


def fp32_envelopes(desc, b, K, B="un", solver="ba", draws=3, seed=0, basis="f64"):
    """How far FP32 arithmetic may move the oracle's K-th GMRES iterate.

    Each operator output of the oracle's solve is multiplied by
    (1 + c u 2^-24), u uniform on [-1, 1] per entry, with c = sqrt(L) for L
    the mean number of terms per row of A (the random-walk size of FP32
    accumulation over L products).  Returns the largest relative distance
    of the perturbed iterate from the unperturbed one over a few seeded
    draws.  Problems whose exact iterate amplifies perturbations (noisy data
    at 20-30 iterations, where the Krylov vectors grow nearly dependent)
    move by 1e-4..1e-3 here; a GPU iterate is held to a small multiple of
    this envelope rather than to a fixed tolerance.  Returns (iterate
    envelope, residual envelope), the second being the largest move of any
    entry of the residual history relative to that entry: a residual far
    below the first one carries the iterate's perturbation magnified by
    their ratio."""
    import oracle
    b = np.asarray(b, np.float64).reshape(-1)
    c = float(np.sqrt(oracle.count_A_updates(desc) / desc.n_rays))
    rng = np.random.default_rng(seed)
    A = lambda v: np.asarray(oracle.project_A(desc, v.reshape(desc.vol_shape))).reshape(-1)
    Bop = oracle.back_projector(desc, B)
    Bf = lambda q: np.asarray(Bop(q.reshape(desc.sino_shape))).reshape(-1)
    if solver == "ba":
        r0 = oracle.ba_gmres(desc, b, K, B=B, basis=basis)
    else:
        r0 = oracle.ab_gmres(desc, b, K, B=B)
    ref = r0.x.reshape(-1)
    rres = np.asarray(r0.res, np.float64)
    worst, worst_res = 0.0, 0.0
    for _ in range(draws):
        p = lambda v: v * (1.0 + c * 2.0 ** -24 * rng.uniform(-1.0, 1.0, v.shape))
        if solver == "ba":
            co, W, res, done, _ = oracle.gmres(lambda v: p(Bf(p(A(v)))), p(Bf(b)), K, basis=basis)
            x = W[:done].T @ co
        else:
            co, W, res, done, _ = oracle.gmres(lambda v: p(A(p(Bf(v)))), b, K)
            x = p(Bf(W[:done].T @ co))
        worst = max(worst, float(np.linalg.norm(x - ref) / np.linalg.norm(ref)))
        res = np.asarray(res, np.float64)
        if res.shape == rres.shape:
            worst_res = max(worst_res, float(np.max(np.abs(res - rres) / np.maximum(rres, 1e-300))))
        else:
            worst_res = float("inf")
    return worst, worst_res
