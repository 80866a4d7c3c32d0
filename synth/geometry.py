"""Plain geometry descriptors (data only).

The conventions these numbers refer to (image centring, detector centring,
view angles, source and detector placement) are stated in the C header
``include/ct.h`` and implemented independently by the HIP library and by the
CPU oracle.  Nothing here computes a ray or a weight.
"""

from dataclasses import dataclass, field
from typing import Optional, Sequence

PARALLEL_2D = 0
CONE_3D = 1


@dataclass(frozen=True)
class GeometryDesc:
    kind: int                 # PARALLEL_2D or CONE_3D
    nx: int
    ny: int
    nz: int                   # 1 for 2D
    voxel: float              # isotropic voxel (pixel) size
    n_views: int
    nu: int                   # detector columns (bins)
    nv: int                   # detector rows, 1 for 2D
    du: float                 # detector pitch along u
    dv: float                 # detector pitch along v (ignored in 2D)
    sod: float = 0.0          # source to isocentre (cone only)
    sdd: float = 0.0          # source to detector (cone only)
    angles: Optional[Sequence[float]] = field(default=None)  # None -> uniform set
    projector: int = 0        # forward model: 0 Joseph, 1 line intersection (Siddon)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_rays(self) -> int:
        return self.n_views * self.nv * self.nu

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def sino_shape(self):
        return (self.n_views, self.nv, self.nu)


def parallel2d(n: int, n_views: int, n_bins: int, voxel: float = 1.0,
               du: float = 1.0, angles=None, projector: int = 0) -> GeometryDesc:
    return GeometryDesc(PARALLEL_2D, n, n, 1, float(voxel), int(n_views),
                        int(n_bins), 1, float(du), 1.0, 0.0, 0.0,
                        None if angles is None else tuple(float(a) for a in angles),
                        int(projector))


def cone3d(n: int, n_views: int, n_det: int, voxel: float = 1.0,
           sod_factor: float = 4.0, sdd_factor: float = 8.0,
           pitch: Optional[float] = None, angles=None, nz: Optional[int] = None,
           nv: Optional[int] = None, projector: int = 0) -> GeometryDesc:
    """Circular cone beam with SOD and SDD given as multiples of the volume
    width N*voxel.  The default detector pitch is one voxel seen at the
    isocentre, i.e. voxel*SDD/SOD."""
    width = n * voxel
    sod = sod_factor * width
    sdd = sdd_factor * width
    if pitch is None:
        pitch = voxel * sdd / sod
    return GeometryDesc(CONE_3D, n, n, n if nz is None else nz, float(voxel),
                        int(n_views), int(n_det), int(n_det if nv is None else nv),
                        float(pitch), float(pitch), float(sod), float(sdd),
                        None if angles is None else tuple(float(a) for a in angles),
                        int(projector))
