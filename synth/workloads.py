"""The five synthetic workloads, with their seeds.

Each builder returns geometry plus phantom and noise draws only.  Turning a
phantom into data (b = A x_true plus noise) needs the forward projector, so
callers do that step with the projector they are testing or timing.

W1  2D parallel beam, 64x64, 90 views over 180 deg, 96 unit bins, 10 ellipses.
W2  3D circular cone beam, 128^3, 180 views over 360 deg, 192x192 detector,
    SOD = 4 N, SDD = 8 N (voxel 1), 12 ellipsoids.
W3  3D cone beam, 256^3, 360 views, 384x384 detector, same ratios, ellipsoids
    plus 5 % smoothed Gaussian texture, Poisson data at 1e5 photons per ray.
W4  batch of four 128^3 volumes in the W2 geometry (autograd check).
W5  64 independent 2D slices of seeded uneven sizes.
Paper size: the dimensions of the paper's scanner data (1024 x 1024 x 300
    volume, 180 views over 360 deg, 1088 x 896 detector of 0.278 mm pixels)
    with a synthetic circular geometry of magnification 2 (SOD = 4 W,
    SDD = 8 W) and one voxel per detector pixel at the isocentre.
"""

import math
import numpy as np

from .geometry import parallel2d, cone3d
from .phantoms import (random_ellipses, rasterize_ellipses, random_ellipsoids,
                       rasterize_ellipsoids, smooth_texture, gaussian_noise)


def w1_geometry():
    return parallel2d(64, 90, 96)


def w1_phantom(seed: int = 101):
    g = w1_geometry()
    ells = random_ellipses(seed, 10, g.nx * g.voxel)
    return rasterize_ellipses(ells, g.nx, g.voxel)


def w2_geometry(n: int = 128, views: int = 180):
    return cone3d(n, views, int(1.5 * n))


def w2_phantom(seed: int = 201, n: int = 128) -> np.ndarray:
    ells = random_ellipsoids(seed, 12, float(n))
    return rasterize_ellipsoids(ells, n, 1.0, dtype=np.float32)


def w3_geometry(n: int = 256, views: int = 360):
    return cone3d(n, views, int(1.5 * n))


def w3_phantom(seed: int = 301, texture_seed: int = 302, n: int = 256) -> np.ndarray:
    """Ellipsoids plus texture: smoothed white noise (sigma 2 voxels) with a
    standard deviation of 5 % of the phantom mean over its support, added
    inside the support and clipped at zero."""
    ells = random_ellipsoids(seed, 12, float(n))
    vol = rasterize_ellipsoids(ells, n, 1.0, dtype=np.float32)
    support = vol > 0
    mean = float(vol[support].mean()) if support.any() else 0.0
    tex = smooth_texture(texture_seed, vol.shape, 2.0)
    vol = vol + np.where(support, (0.05 * mean) * tex, 0.0).astype(np.float32)
    np.maximum(vol, 0.0, out=vol)
    return vol.astype(np.float32)


def w4_phantoms(n: int = 128):
    return [w2_phantom(401 + i, n) for i in range(4)]


def w5_slices(seed: int = 501, count: int = 64):
    """List of (geometry, phantom seed, noise seed) for the uneven batch."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice([128, 192, 256, 384, 512], size=count)
    views = rng.choice([90, 180, 360], size=count)
    out = []
    for i in range(count):
        n = int(sizes[i])
        g = parallel2d(n, int(views[i]), int(math.ceil(1.5 * n)))
        out.append((g, 510 + i, 600 + i))
    return out


def w5_phantom(g, seed: int) -> np.ndarray:
    ells = random_ellipses(seed, 10, g.nx * g.voxel)
    return rasterize_ellipses(ells, g.nx, g.voxel)


def relative_gaussian_noise(clean: np.ndarray, level: float, seed: int) -> np.ndarray:
    """e = level * ||clean|| * eta / ||eta||, eta ~ N(0, I)."""
    eta = gaussian_noise(seed, clean.size).reshape(clean.shape)
    return level * np.linalg.norm(clean) * eta / np.linalg.norm(eta)


def paper_geometry():
    pitch = 0.278
    voxel = pitch / 2.0
    return cone3d(1024, 180, 1088, voxel=voxel, sod_factor=4.0, sdd_factor=8.0, pitch=pitch,
                  nz=300, nv=896)


def paper_phantom_ellipsoids(seed: int = 701):
    """12 random ellipsoids over 0.7 of the volume width, so that they stay
    inside the field of view of the 1088-pixel detector."""
    g = paper_geometry()
    return random_ellipsoids(seed, 12, 0.7 * g.nx * g.voxel)
