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


# small geometries spanning several tiles with ragged tails
SMALL_GEOMS = {
    "w1_2d_64": parallel2d(64, 90, 96),
    "ragged_2d": GeometryDesc(PARALLEL_2D, 37, 29, 1, 0.9, 50, 61, 1, 1.1, 1.0),
    "explicit_angles_2d": parallel2d(40, 33, 70, angles=[0.1 + 0.093 * p for p in range(33)]),
    "cone_24": cone3d(24, 20, 36),
    "ragged_cone": GeometryDesc(CONE_3D, 33, 30, 17, 1.0, 13, 45, 29, 1.7, 2.3, 140.0, 290.0),
    "cone_45deg_views": cone3d(20, 8, 30),   # views at multiples of 45 deg
}
