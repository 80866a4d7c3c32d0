"""Seeded phantoms and noise draws (input data only).

Readings used for the workloads (the paper demonstrates its method on a
scanner data set that is not available; these synthetic phantoms stand in):

* ellipse / ellipsoid full axis lengths U[0.05, 0.4] * FOV (semi-axes half
  that), centres U[-0.3, 0.3] * FOV per coordinate, densities U[0, 1] and
  additive where objects overlap;
* 2D rotation U[0, pi); 3D rotation uniform over SO(3) from the QR
  factorisation of a Gaussian matrix with the sign of R's diagonal fixed;
* rasterisation by point sampling at voxel centres, optionally supersampled;
* ``profile="smooth"`` replaces the constant density by (1 - rho^2)^2, rho the
  normalised radius, used for convergence-order checks.
"""

import numpy as np


def _centres(n: int, voxel: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * voxel


# --------------------------------------------------------------------- 2D
def random_ellipses(seed: int, count: int, fov: float):
    """Return a list of dicts (cx, cy, a, b, phi, rho) with semi-axes a, b."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        cx, cy = rng.uniform(-0.3, 0.3, size=2) * fov
        a, b = 0.5 * rng.uniform(0.05, 0.4, size=2) * fov
        phi = rng.uniform(0.0, np.pi)
        rho = rng.uniform(0.0, 1.0)
        out.append(dict(cx=float(cx), cy=float(cy), a=float(a), b=float(b),
                        phi=float(phi), rho=float(rho)))
    return out


def _ellipse_unit_radius2(ell, X, Y):
    c, s = np.cos(ell["phi"]), np.sin(ell["phi"])
    dx, dy = X - ell["cx"], Y - ell["cy"]
    # coordinates in the ellipse frame, scaled to the unit disk
    u = (c * dx + s * dy) / ell["a"]
    v = (-s * dx + c * dy) / ell["b"]
    return u * u + v * v


def rasterize_ellipses(ells, n: int, voxel: float, profile: str = "uniform",
                       supersample: int = 1) -> np.ndarray:
    """Image [n][n] (row = y index, column = x index), float64."""
    img = np.zeros((n, n), dtype=np.float64)
    ss = int(supersample)
    offs = ((np.arange(ss) + 0.5) / ss - 0.5) * voxel
    xc = _centres(n, voxel)
    for oy in offs:
        for ox in offs:
            X = (xc + ox)[None, :]
            Y = (xc + oy)[:, None]
            for e in ells:
                r2 = _ellipse_unit_radius2(e, X, Y)
                if profile == "uniform":
                    img += e["rho"] * (r2 <= 1.0)
                else:
                    img += e["rho"] * np.where(r2 < 1.0, (1.0 - r2) ** 2, 0.0)
    return img / (ss * ss)


# --------------------------------------------------------------------- 3D
def _random_rotation(rng) -> np.ndarray:
    g = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_ellipsoids(seed: int, count: int, fov: float):
    """List of dicts: centre (3,), semi (3,), R (3x3, columns = axes), rho."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        c = rng.uniform(-0.3, 0.3, size=3) * fov
        semi = 0.5 * rng.uniform(0.05, 0.4, size=3) * fov
        R = _random_rotation(rng)
        rho = rng.uniform(0.0, 1.0)
        out.append(dict(centre=c, semi=semi, R=R, rho=float(rho)))
    return out


def rasterize_ellipsoids(ells, n: int, voxel: float, profile: str = "uniform",
                         supersample: int = 1, nz: int = None,
                         dtype=np.float64) -> np.ndarray:
    """Volume [nz][ny][nx] (x fastest), point-sampled at voxel centres."""
    nz = n if nz is None else nz
    vol = np.zeros((nz, n, n), dtype=dtype)
    ss = int(supersample)
    offs = ((np.arange(ss) + 0.5) / ss - 0.5) * voxel
    xc = _centres(n, voxel)
    zc = _centres(nz, voxel)
    for e in ells:
        # bounding box of the ellipsoid in voxel index space
        ext = np.sqrt(((e["R"] * e["semi"][None, :]) ** 2).sum(axis=1))
        lo = np.floor((e["centre"] - ext) / voxel + 0.5 * (np.array([n, n, nz]) - 1)) - 1
        hi = np.ceil((e["centre"] + ext) / voxel + 0.5 * (np.array([n, n, nz]) - 1)) + 2
        ix0, iy0, iz0 = [int(max(0, v)) for v in lo]
        ix1, iy1, iz1 = [int(min(m, v)) for v, m in zip(hi, (n, n, nz))]
        if ix0 >= ix1 or iy0 >= iy1 or iz0 >= iz1:
            continue
        Rt = e["R"].T
        acc = np.zeros((iz1 - iz0, iy1 - iy0, ix1 - ix0), dtype=np.float64)
        for oz in offs:
            for oy in offs:
                for ox in offs:
                    Z = (zc[iz0:iz1] + oz)[:, None, None] - e["centre"][2]
                    Y = (xc[iy0:iy1] + oy)[None, :, None] - e["centre"][1]
                    X = (xc[ix0:ix1] + ox)[None, None, :] - e["centre"][0]
                    # coordinates along the ellipsoid axes, scaled to the unit ball
                    u = (Rt[0, 0] * X + Rt[0, 1] * Y + Rt[0, 2] * Z) / e["semi"][0]
                    v = (Rt[1, 0] * X + Rt[1, 1] * Y + Rt[1, 2] * Z) / e["semi"][1]
                    w = (Rt[2, 0] * X + Rt[2, 1] * Y + Rt[2, 2] * Z) / e["semi"][2]
                    r2 = u * u + v * v + w * w
                    if profile == "uniform":
                        acc += (r2 <= 1.0)
                    else:
                        acc += np.where(r2 < 1.0, (1.0 - r2) ** 2, 0.0)
        vol[iz0:iz1, iy0:iy1, ix0:ix1] += (e["rho"] / ss ** 3) * acc
    return vol


def rasterize_ellipsoids_torch(ells, n: int, voxel: float, nz: int, device):
    """The uniform-profile rasterisation of rasterize_ellipsoids (point
    samples at voxel centres, additive densities), evaluated with torch on
    `device` slab by slab for volumes too large for the numpy version.
    Returns a float32 tensor [nz][n][n]."""
    import torch
    vol = torch.zeros((nz, n, n), dtype=torch.float32, device=device)
    xc = torch.as_tensor(_centres(n, voxel), dtype=torch.float64, device=device)
    zc = torch.as_tensor(_centres(nz, voxel), dtype=torch.float64, device=device)
    for e in ells:
        ext = np.sqrt(((e["R"] * e["semi"][None, :]) ** 2).sum(axis=1))
        lo = np.floor((e["centre"] - ext) / voxel + 0.5 * (np.array([n, n, nz]) - 1)) - 1
        hi = np.ceil((e["centre"] + ext) / voxel + 0.5 * (np.array([n, n, nz]) - 1)) + 2
        ix0, iy0, iz0 = [int(max(0, v)) for v in lo]
        ix1, iy1, iz1 = [int(min(m, v)) for v, m in zip(hi, (n, n, nz))]
        if ix0 >= ix1 or iy0 >= iy1 or iz0 >= iz1:
            continue
        Rt = e["R"].T
        X = (xc[ix0:ix1] - e["centre"][0])[None, :]
        Y = (xc[iy0:iy1] - e["centre"][1])[:, None]
        for z0 in range(iz0, iz1, 16):
            z1 = min(z0 + 16, iz1)
            Z = (zc[z0:z1] - e["centre"][2])[:, None, None]
            u = (Rt[0, 0] * X + Rt[0, 1] * Y)[None] + Rt[0, 2] * Z
            v = (Rt[1, 0] * X + Rt[1, 1] * Y)[None] + Rt[1, 2] * Z
            w = (Rt[2, 0] * X + Rt[2, 1] * Y)[None] + Rt[2, 2] * Z
            r2 = (u / e["semi"][0]) ** 2 + (v / e["semi"][1]) ** 2 + (w / e["semi"][2]) ** 2
            vol[z0:z1, iy0:iy1, ix0:ix1] += float(e["rho"]) * (r2 <= 1.0).float()
    return vol


# ------------------------------------------------------------ noise draws
def smooth_texture(seed: int, shape, sigma: float = 2.0) -> np.ndarray:
    """White Gaussian noise smoothed by a Gaussian of ``sigma`` voxels and
    renormalised to unit standard deviation (float32)."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape, dtype=np.float32)
    s = gaussian_filter(w, sigma=sigma, mode="constant")
    s /= max(float(s.std()), 1e-30)
    return s


def gaussian_noise(seed: int, size: int) -> np.ndarray:
    """eta ~ N(0, I), float64; the caller scales it to a relative level."""
    return np.random.default_rng(seed).standard_normal(size)


def poisson_log_counts(seed: int, line_integrals: np.ndarray, photons: float) -> np.ndarray:
    """Measurement model for log-transformed transmission data:
    counts ~ Poisson(photons * exp(-l)), b = -ln(max(counts, 1) / photons)."""
    rng = np.random.default_rng(seed)
    lam = photons * np.exp(-np.asarray(line_integrals, dtype=np.float64))
    counts = rng.poisson(lam).astype(np.float64)
    return -np.log(np.maximum(counts, 1.0) / photons)
