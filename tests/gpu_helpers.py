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


def fp32_envelope(desc, b, K, B="un", solver="ba", draws=3, seed=0, basis="f64"):
    """How far FP32 arithmetic may move the oracle's K-th GMRES iterate.

    Each operator output of the oracle's solve is multiplied by
    (1 + c u 2^-24), u uniform on [-1, 1] per entry, with c = sqrt(L) for L
    the mean number of terms per row of A (the random-walk size of FP32
    accumulation over L products).  Returns the largest relative distance
    of the perturbed iterate from the unperturbed one over a few seeded
    draws.  Problems whose exact iterate amplifies perturbations (noisy data
    at 20-30 iterations, where the Krylov vectors grow nearly dependent)
    move by 1e-4..1e-3 here; a GPU iterate is held to a small multiple of
    this envelope rather than to a fixed tolerance."""
    import oracle
    b = np.asarray(b, np.float64).reshape(-1)
    c = float(np.sqrt(oracle.count_A_updates(desc) / desc.n_rays))
    rng = np.random.default_rng(seed)
    A = lambda v: np.asarray(oracle.project_A(desc, v.reshape(desc.vol_shape))).reshape(-1)
    Bop = oracle.back_projector(desc, B)
    Bf = lambda q: np.asarray(Bop(q.reshape(desc.sino_shape))).reshape(-1)
    if solver == "ba":
        ref = oracle.ba_gmres(desc, b, K, B=B, basis=basis).x.reshape(-1)
    else:
        ref = oracle.ab_gmres(desc, b, K, B=B).x.reshape(-1)
    worst = 0.0
    for _ in range(draws):
        p = lambda v: v * (1.0 + c * 2.0 ** -24 * rng.uniform(-1.0, 1.0, v.shape))
        if solver == "ba":
            co, W, _, done, _ = oracle.gmres(lambda v: p(Bf(p(A(v)))), p(Bf(b)), K, basis=basis)
            x = W[:done].T @ co
        else:
            co, W, _, done, _ = oracle.gmres(lambda v: p(A(p(Bf(v)))), b, K)
            x = p(Bf(W[:done].T @ co))
        worst = max(worst, float(np.linalg.norm(x - ref) / np.linalg.norm(ref)))
    return worst
