"""Write tests/golden/cgls_fp32_spread.json: how far FP32 storage of the CGLS
vectors moves the oracle's own CGLS(A^T) iterates on the 128^3 cone-beam
workload (noiseless data, 50 iterations), computed with the FP64 oracle's
operators only.

CGLS (Sec. I, Eq. 2) is a short recurrence: each step builds on the previous
vectors, so rounding them to FP32 changes later iterates far more than it
changes one operator application.  The spread is the largest, over two
runs, of the relative distance of the FP32-vector iterate x_50 from the FP64
one, and of the largest per-step relative distance of the data residual
||b - A x_k||:
  run 1: every vector (x, r, s, p) and every operator output rounded to
         FP32 after each update, scalars in FP64;
  run 2: as run 1, with each operator output also multiplied by
         (1 + c u 2^-24), u uniform on [-1, 1] per entry (seed 0) and c the
         square root of the mean number of samples per ray, the random-walk
         size of FP32 accumulation.
The GPU tests hold the GPU's CGLS to three times these figures.

    python tests/golden/make_cgls_spread.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import workloads  # noqa: E402


def f32(v):
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float64)


def cgls_rounded(desc, b, iters, perturb=None):
    A = lambda v: f32(perturb(oracle.project_A(desc, v)) if perturb else oracle.project_A(desc, v))
    AT = lambda v: f32(perturb(oracle.backproject_AT(desc, v)) if perturb else oracle.backproject_AT(desc, v))
    x = np.zeros(desc.n_vox)
    r = b.copy()
    s = AT(r)
    p = s.copy()
    gamma = float(s @ s)
    res = [float(np.linalg.norm(r))]
    for _ in range(iters):
        q = A(p)
        alpha = gamma / float(q @ q)
        x = f32(x + alpha * p)
        r = f32(r - alpha * q)
        s = AT(r)
        gamma_new = float(s @ s)
        p = f32(s + (gamma_new / gamma) * p)
        gamma = gamma_new
        res.append(float(np.linalg.norm(r)))
    return x, np.array(res)


def main():
    K = 50
    desc = workloads.w2_geometry()
    vol = workloads.w2_phantom()
    b = f32(oracle.project_A(desc, vol))
    ref = oracle.cgls(desc, b, K, B="AT")
    rx = np.asarray(ref.x)
    rres = np.array(ref.res)
    c = float(np.sqrt(oracle.count_A_updates(desc) / desc.n_rays))
    rng = np.random.default_rng(0)
    pert = lambda v: v * (1.0 + c * 2.0 ** -24 * rng.uniform(-1.0, 1.0, v.shape))
    out = {"x": 0.0, "res": 0.0, "runs": []}
    for name, pf in (("fp32 vectors", None), ("fp32 vectors + operator perturbation", pert)):
        x, res = cgls_rounded(desc, b, K, pf)
        ex = float(np.linalg.norm(x - rx) / np.linalg.norm(rx))
        er = float(np.max(np.abs(res - rres) / rres))
        print(name, "x %.3e  residual %.3e" % (ex, er), flush=True)
        out["runs"].append({"run": name, "x": ex, "res": er})
        out["x"] = max(out["x"], ex)
        out["res"] = max(out["res"], er)
    out["iters"] = K
    out["residual_first_last"] = [float(rres[0]), float(rres[-1])]
    path = os.path.join(HERE, "cgls_fp32_spread.json")
    with open(path, "w") as f:
        json.dump({"w2_cgls_AT_50": out}, f, indent=1)


if __name__ == "__main__":
    main()
