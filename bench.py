"""Benchmark: BA-GMRES iterations/s on the 256^3 cone-beam workload.

One step = one BA-GMRES solve (K = 30 iterations, B = B_un F, the
ramp-filtered voxel-driven back-projector) from b resident in HBM to x in
HBM, including the final host copy of the residual history.  The timed
steps run without kernel timing; the per-kernel times come from a separate
pass with the library's event pairs.

Workload (synthetic stand-in for the paper's scanner data): 256^3 volume of
12 random ellipsoids plus 5 % smoothed Gaussian texture; circular cone beam,
360 views over 360 deg, 384 x 384 detector at one voxel per pixel at the
isocentre, SOD = 4 N, SDD = 8 N; data from the FP64 oracle's projector
(from the GPU's with --no-cpu), scaled so the largest line integral is 4,
Poisson counts at 1e5 photons per ray, negative log.

Prints one JSON line with the throughput, the roofline position of the
dominant kernel, the FP64 CPU oracle timed on a bounded sample of the same
workload and the distance of the GPU iterate from the oracle's, plus the
extra legs (FP16 data storage, the matched transpose, the per-iteration
curves of Sec. III / Fig. 2 on the 128^3 workload, FP16 basis, the
line-intersection model, the batched 2D slices).

    python bench.py [--steps K] [--warmup W] [--sino-dtype f32|f16] [--no-cpu] ...
"""

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ITERS = 30
PEAK_FP32_VECTOR = 157.3e12     # MI355X published FP32 vector peak, FLOP/s
PEAK_HBM = 8.0e12               # bytes/s
# algorithmic work per unit, counting each step of a sample as one
# operation: a Joseph sample is 2 coordinates, 2 fractions, 3 linear
# interpolations and an accumulate (about 10 FLOP); a voxel-driven update a
# coordinate, a fraction, 3 interpolations and a weighted accumulate (about
# 8).  Counting an FMA as two and an interpolation as a subtract plus an FMA
# gives 16 and 14 instead, and fractions 1.6 and 1.75 times higher.
FLOP_PER_A_UPDATE = 10.0
FLOP_PER_B_UPDATE = 8.0
# HBM traffic of one projector launch on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE passes over this benchmark, each scaled by what
# the counter reads for a 256 MiB copy (FETCH x2.0, WRITE x1.0); valid only
# for the projector source and launch set-up it was measured on (hash of
# their text)
A_TRAFFIC_BYTES = 6816395059
A_TRAFFIC_SRC = "f19e6b0276162d7f"


_T_START = time.perf_counter()


def log(*a):
    print("[%6.1f s]" % (time.perf_counter() - _T_START), *a, file=sys.stderr, flush=True)


def phantom_scaled_data(vol, clean, seed=303):
    """b = -log of Poisson counts at 1e5 photons of the line integrals scaled
    so that the largest is 4; returns (b as FP32, the attenuation that makes
    exactly those line integrals)."""
    from synth.phantoms import poisson_log_counts
    mu = 4.0 / float(clean.max())
    b = poisson_log_counts(seed, clean * mu, 1e5).astype(np.float32)
    return b, vol * mu


def projector_src_hash():
    """Hash of the projector's kernel source and of its launch set-up (view
    groups, workgroup order): the stored traffic figure belongs to it."""
    import hashlib
    path = os.path.join(ROOT, "paper_2201_07408_amd", "csrc", "ct_projectors.hip")
    src = open(path).read()
    parts = []
    for start, end in (("struct RaySetup {", "constexpr int kZC = 16;"),
                       ("constexpr double kLlcBytes", "int launch_col_table(")):
        a, b = src.find(start), src.find(end)
        if a < 0 or b < a:
            return None
        parts.append(src[a:b])
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


# ------------------------------------------------------------ CPU oracle leg
# Everything that runs the FP64 oracle: the data of the 256^3 and 128^3
# workloads from the oracle's own projector (so that no GPU operator shapes
# the right-hand sides both sides solve), the oracle's 256^3 iterate the GPU
# is compared with, and the oracle timed on the host's threads.
def oracle_data(desc3, vol3, desc2, vol2):
    import oracle
    t0 = time.perf_counter()
    clean3 = np.asarray(oracle.project_A(desc3, vol3))
    t_a3 = time.perf_counter() - t0
    clean2 = np.asarray(oracle.project_A(desc2, vol2))
    return clean3, clean2, t_a3


def cpu_baseline(desc3, b3, K=2):
    """FP64 oracle BA-GMRES (B_un F) on the 256^3 workload, K iterations on
    all of the host's threads: the iterate the GPU's is compared with, and
    the oracle's rate (the start vector costs about half an iteration, so
    seconds per iteration are the time over K + 0.5)."""
    import oracle
    t0 = time.perf_counter()
    ref = oracle.ba_gmres(desc3, b3.astype(np.float64), K, B="ramp")
    dt = time.perf_counter() - t0
    per_iter = dt / (ref.iters_done + 0.5)
    out = {"value": 1.0 / per_iter, "unit": "iters/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": "FP64 oracle BA-GMRES (B_un F), %d iterations on the full 256^3 workload (360 views, "
                     "384x384 detector) on %d host threads; %.1f s of CPU work, seconds per iteration "
                     "= time / (K + 0.5)" % (K, oracle.num_threads(), dt)}
    return out, ref


def cpu_small_configs(desc1, b1, desc2, b2):
    """The oracle's BA-GMRES (B_un) rate on the 64^2 workload (30
    iterations), the 128^3 workload (2 iterations) and one 256^2 slice of
    the batched 2D workload, at one thread and at all threads; at one thread
    the 128^3 solve runs on every 10th view and its seconds are scaled by 10
    (operator cost is linear in views), and the slice runs 10 iterations."""
    import oracle
    from synth.geometry import GeometryDesc
    nthr = oracle.num_threads()
    out = {"threads_all": nthr}

    def rate(desc, b, K):
        t0 = time.perf_counter()
        r = oracle.ba_gmres(desc, b, K, B="un")
        return (r.iters_done + 0.5) / (time.perf_counter() - t0)

    try:
        for name, th in (("1_thread", 1), ("all_threads", nthr)):
            oracle.set_threads(th)
            out.setdefault("C1_64x64_K30_iters_per_s", {})[name] = rate(desc1, b1, 30)
        oracle.set_threads(nthr)
        out.setdefault("C2_128cube_iters_per_s", {})["all_threads"] = rate(desc2, b2, 2)
        sub = 10
        angles = [2 * math.pi * p / desc2.n_views for p in range(0, desc2.n_views, sub)]
        gs = GeometryDesc(desc2.kind, desc2.nx, desc2.ny, desc2.nz, desc2.voxel, len(angles), desc2.nu,
                          desc2.nv, desc2.du, desc2.dv, desc2.sod, desc2.sdd, tuple(angles))
        bs = np.ascontiguousarray(b2.reshape(desc2.sino_shape)[::sub])
        oracle.set_threads(1)
        out["C2_128cube_iters_per_s"]["1_thread"] = rate(gs, bs, 2) / sub
        out["C2_128cube_iters_per_s"]["1_thread_sample"] = "every %dth view, seconds scaled by %d" % (sub, sub)
        # one slice of the batched 2D workload (256^2, 180 views, 384 bins,
        # 1 % noise), as the batch solves it (B_un, 40 iterations) on all
        # threads and for 10 iterations on one thread
        from synth import workloads
        g5, ps5, ns5 = next(t for t in workloads.w5_slices() if t[0].nx == 256 and t[0].n_views == 180)
        c5 = np.asarray(oracle.project_A(g5, workloads.w5_phantom(g5, ps5)))
        b5 = c5 + workloads.relative_gaussian_noise(c5, 0.01, ns5)
        s5 = out.setdefault("C5_slice_256x256_180views_iters_per_s", {})
        s5["1_thread"] = rate(g5, b5, 10)
        oracle.set_threads(nthr)
        s5["all_threads"] = rate(g5, b5, 40)
        s5["sample"] = "one slice of the 64-slice batch; 10 iterations at one thread, 40 at all threads"
    finally:
        oracle.set_threads(nthr)
    return out


def sampled_errors(desc, ct, g, torch, x_phantom):
    """Relative error of the GPU operators against the FP64 oracle on sampled
    rays / voxels of the benchmark workload."""
    import oracle
    rng = np.random.default_rng(11)
    x = torch.from_numpy(np.ascontiguousarray(x_phantom, dtype=np.float32)).cuda()
    y = ct.ct_project_A(g, x)
    yh = y.double().cpu().numpy().reshape(-1)
    rays = rng.choice(desc.n_rays, size=1500, replace=False)
    ra = oracle.project_A_rays(desc, x.double().cpu().numpy(), rays)
    ea = float(np.linalg.norm(yh[rays] - ra) / np.linalg.norm(ra))
    xb = ct.ct_backproject_B(g, y, ramp=True).double().cpu().numpy().reshape(-1)
    vox = rng.choice(desc.n_vox, size=1500, replace=False)
    fy = oracle.ramp(desc, y.float().cpu().numpy())
    rb = oracle.backproject_Bun_voxels(desc, fy, vox)
    eb = float(np.linalg.norm(xb[vox] - rb) / np.linalg.norm(rb))
    return {"A_sampled": ea, "B_FBP_sampled": eb}


# ------------------------------------------------------------------ GPU legs
def gpu_data(ct, g, torch, vol):
    """Line integrals of the phantom from the GPU's projector (used only when
    the oracle leg is switched off)."""
    x = torch.from_numpy(vol).cuda()
    return ct.ct_project_A(g, x).double().cpu().numpy().reshape(-1)


def bench_f16_data(ct, torch, g, b, x_phantom, x32, steps=3):
    """The headline solve with the solver's projections stored in FP16
    (FP32 arithmetic): rate, distance from the FP32-storage iterate and
    image RMSE of both."""
    x_ref = torch.from_numpy(np.ascontiguousarray(x_phantom, dtype=np.float32)).cuda()
    rmse = lambda v: float(torch.sqrt(torch.mean((v.double() - x_ref.double()) ** 2)))
    ct.ct_ba_gmres(g, b, ITERS, B="ramp", sino_dtype=torch.float16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for _ in range(steps):
        r = ct.ct_ba_gmres(g, b, ITERS, B="ramp", sino_dtype=torch.float16)
        done += r.iters_done
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"iters_per_s": done / dt, "data_bytes_per_projection": 2 * g.n_rays,
            "rel_diff_vs_fp32_storage": float(torch.linalg.vector_norm(r.x - x32) / torch.linalg.vector_norm(x32)),
            "image_rmse": rmse(r.x), "image_rmse_fp32_storage": rmse(x32),
            "residual_at_30": r.res[-1], "residual_at_30_fp32_storage": None}


def bench_fig2(ct, torch, clean2, vol2, K=50):
    """The comparison of Sec. III / Fig. 2 on the 128^3 workload: the data
    residual ||A x_k - b|| (and the data RMSE, that norm over sqrt(m)) of
    CGLS with the unmatched B_un, CGLS with A^T, BA-GMRES with B_un and
    BA-GMRES with B_FBP, for k = 0..K, on noiseless data and with 1 %
    Gaussian noise (seed 202).  Reported, not asserted: on this synthetic
    problem the unmatched CGLS need not diverge within K."""
    from synth import workloads
    desc = workloads.w2_geometry()
    g = ct.Geometry(desc)
    x_ref = torch.from_numpy(np.ascontiguousarray(vol2, dtype=np.float32)).cuda()
    sm = math.sqrt(desc.n_rays)
    out = {"workload": "128^3 cone beam, 180 views, 192x192 detector, 12 ellipsoids; %d iterations" % K,
           "every": 5}
    for name, noise in (("noiseless", 0.0), ("noise_1pct", 0.01)):
        y = clean2 + (workloads.relative_gaussian_noise(clean2, noise, 202) if noise > 0 else 0.0)
        b = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).cuda()
        curves = {}
        t0 = time.perf_counter()
        for B, label in (("un", "CGLS_B_un"), ("AT", "CGLS_AT")):
            r = ct.ct_cgls(g, b, K, B=B)
            img = float(torch.sqrt(torch.mean((r.x.double() - x_ref.double()) ** 2)))
            curves[label] = {"data_residual": [round(v, 6) for v in r.res[::5]],
                             "min_at": int(np.argmin(r.res)), "last_over_min": r.res[-1] / min(r.res),
                             "image_rmse_at_K": img}
        for B, label in (("un", "BA_GMRES_B_un"), ("ramp", "BA_GMRES_B_FBP")):
            r = ct.ct_ba_gmres_monitor(g, b, K, B=B, x_ref=x_ref)
            curves[label] = {"data_residual": [round(v, 6) for v in r.data_res[::5]],
                             "min_at": int(np.nanargmin(r.data_res)),
                             "last_over_min": r.data_res[-1] / np.nanmin(r.data_res),
                             "image_rmse": [round(v, 7) for v in r.img_rmse[::5]],
                             "min_image_rmse_at": int(np.nanargmin(r.img_rmse))}
        torch.cuda.synchronize()
        curves["data_rmse_divisor"] = sm
        curves["s_all_curves"] = time.perf_counter() - t0
        out[name] = curves
    return out


def bench_batched(ct, torch, reps=3):
    """64 uneven 2D slices (N in {128..512}, 90/180/360 views, ceil(1.5 N)
    bins, ellipse phantoms, 1 % noise), BA-GMRES(B_un) for 40 iterations
    each: one batched solve (hipGraph replay) against the same 64 solves
    one after another.  Both are warmed first (every geometry's solver
    workspace exists before the timed passes) and both are timed over the
    same number of repetitions.  Inputs are made with the library's own
    projector."""
    from synth import workloads
    K = 40
    slices = workloads.w5_slices()
    geoms, bs = [], []
    for d, pseed, nseed in slices:
        g = ct.Geometry(d)
        x = torch.from_numpy(workloads.w5_phantom(d, pseed).astype(np.float32)).cuda()
        y = ct.ct_project_A(g, x).double().cpu().numpy()
        y = y + workloads.relative_gaussian_noise(y, 0.01, nseed)
        geoms.append(g)
        bs.append(torch.from_numpy(y.astype(np.float32)).cuda())
    out = ct.ct_ba_gmres_batched(geoms, bs, K)          # autotune + graph capture
    seq = [ct.ct_ba_gmres(g, b, K) for g, b in zip(geoms, bs)]   # every workspace allocated
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = ct.ct_ba_gmres_batched(geoms, bs, K)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    done_b = sum(r.iters_done for r in out)
    t0 = time.perf_counter()
    for _ in range(reps):
        seq = [ct.ct_ba_gmres(g, b, K) for g, b in zip(geoms, bs)]
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / reps
    done_s = sum(r.iters_done for r in seq)
    diff = max(float(torch.linalg.norm(r.x - s.x) / torch.linalg.norm(s.x)) for r, s in zip(out, seq))
    graph, a_var, b_var = ct.ct_batched_last_config()
    return {"workload": "64 2D parallel-beam slices, N in {128,192,256,384,512}, 90/180/360 views, "
                        "ceil(1.5N) bins, BA-GMRES(B_un) 40 iterations each",
            "batched_iters_per_s": done_b / tb, "sequential_iters_per_s": done_s / ts,
            "speedup": ts / tb * done_b / max(done_s, 1), "batched_ms": tb * 1e3, "sequential_ms": ts * 1e3,
            "reps_each": reps, "max_rel_diff_x_vs_sequential": diff, "hipgraph": graph,
            "projector_variant": a_var, "backprojector_variant": b_var}


def bench_siddon(ct, torch, lib, steps=2):
    """BA-GMRES (B = B_un F, 30 iterations) on the 256^3 workload with the
    line-intersection forward model (the paper's A) instead of Joseph's:
    data from the same phantom through that projector, Poisson 1e5."""
    import dataclasses
    from synth import workloads
    from synth.phantoms import poisson_log_counts
    desc = dataclasses.replace(workloads.w3_geometry(), projector=1)
    g = ct.Geometry(desc)
    x = torch.from_numpy(workloads.w3_phantom()).cuda()
    ax = ct.ct_project_A(g, x)
    mu = 4.0 / float(ax.max())
    b = torch.from_numpy(poisson_log_counts(303, (ax * mu).double().cpu().numpy().reshape(-1),
                                            1e5).astype(np.float32)).cuda()
    ct.ct_ba_gmres(g, b, ITERS, B="ramp")
    torch.cuda.synchronize()
    lib.ct_profile_reset()
    lib.ct_profile_enable(1)
    t0 = time.perf_counter()
    done = 0
    for _ in range(steps):
        done += ct.ct_ba_gmres(g, b, ITERS, B="ramp").iters_done
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lib.ct_profile_enable(0)
    n_l, t_l = ctypes.c_long(), ctypes.c_double()
    lib.ct_profile_read(b"A", ctypes.byref(n_l), ctypes.byref(t_l))
    t_a = t_l.value / 1e3 / max(n_l.value, 1)
    counts = json.load(open(os.path.join(ROOT, "tests", "golden", "update_counts.json")))["w3_siddon"]
    return {"workload": "as the headline, forward model = line-intersection (Siddon) A",
            "iters_per_s": done / dt, "A_ms_per_launch": t_a * 1e3,
            "A_segments_per_s": counts["A_updates"] / t_a, "A_segments_per_launch": counts["A_updates"]}


def bench_monitor(ct, torch, b, x_phantom, plain_ms):
    """Semi-convergence on the headline workload: the per-iteration image
    RMSE against the attenuation that made the data and the data residual,
    for B = B_un and B = B_un F, and the monitor's cost per iteration."""
    x_ref = torch.from_numpy(np.ascontiguousarray(x_phantom, dtype=np.float32)).cuda()
    g = ct.Geometry(__import__("synth").workloads.w3_geometry())
    out = {}
    for B in ("un", "ramp"):
        ct.ct_ba_gmres_monitor(g, b, ITERS, B=B, x_ref=x_ref)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ct.ct_ba_gmres_monitor(g, b, ITERS, B=B, x_ref=x_ref)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        img = np.array(r.img_rmse)
        k = int(np.nanargmin(img))
        out["B_un" if B == "un" else "B_FBP"] = {
            "min_image_rmse": float(img[k]), "at_iteration": k,
            "image_rmse_at_30": float(img[-1]), "data_residual_at_30": float(r.data_res[-1]),
            "data_residual_at_0": float(r.data_res[0]), "ms_per_solve": dt * 1e3}
    out["monitor_overhead_ms_per_iteration"] = (out["B_FBP"]["ms_per_solve"] - plain_ms) / ITERS
    # the one-shot FDK reconstruction of the same data, for comparison
    xf = ct.ct_fbp(g, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xf = ct.ct_fbp(g, b, out=xf)
    torch.cuda.synchronize()
    fdk_ms = (time.perf_counter() - t0) * 1e3
    out["FDK"] = {"image_rmse": float(torch.sqrt(torch.mean((xf.double() - x_ref.double()) ** 2))),
                  "ms": fdk_ms}
    return out


def bench_basis16(ct, torch, lib, g, b, x_phantom, x32):
    """The Krylov basis stored in FP16 on the headline workload: the full
    30-iteration solve (time, orthogonalisation time, distance from the
    FP32-basis iterate, image RMSE) and restarted BA-GMRES(10) x 3 cycles
    with FP16 and FP32 bases (image RMSE, basis bytes)."""
    import ctypes as C
    x_ref = torch.from_numpy(np.ascontiguousarray(x_phantom, dtype=np.float32)).cuda()
    rmse = lambda x: float(torch.sqrt(torch.mean((x.double() - x_ref.double()) ** 2)))
    n = x_ref.numel()
    out = {"basis_bytes_full_fp32": 4 * n * (ITERS + 1), "basis_bytes_full_fp16": 2 * n * (ITERS + 1),
           "basis_bytes_restart10_fp16": 2 * n * 11}
    ct.ct_ba_gmres(g, b, ITERS, B="ramp", basis_dtype=torch.float16)
    torch.cuda.synchronize()
    lib.ct_profile_reset()
    lib.ct_profile_enable(1)
    t0 = time.perf_counter()
    r = ct.ct_ba_gmres(g, b, ITERS, B="ramp", basis_dtype=torch.float16)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lib.ct_profile_enable(0)
    n_l, t_l = C.c_long(), C.c_double()
    lib.ct_profile_read(b"CGS", C.byref(n_l), C.byref(t_l))
    out["full_fp16"] = {"iters_per_s": r.iters_done / dt, "CGS_ms_per_iteration": t_l.value / max(r.iters_done, 1),
                        "rel_diff_vs_fp32_basis": float(torch.linalg.vector_norm(r.x - x32) /
                                                        torch.linalg.vector_norm(x32)),
                        "image_rmse": rmse(r.x), "image_rmse_fp32_basis": rmse(x32),
                        "residual_at_30": r.res[-1], "residual_at_0": r.res[0]}
    for name, bd in (("restart10x3_fp16", torch.float16), ("restart10x3_fp32", torch.float32)):
        ct.ct_ba_gmres_restarted(g, b, 10, 3, B="ramp", basis_dtype=bd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rr = ct.ct_ba_gmres_restarted(g, b, 10, 3, B="ramp", basis_dtype=bd)
        torch.cuda.synchronize()
        out[name] = {"ms_per_solve": (time.perf_counter() - t0) * 1e3, "image_rmse": rmse(rr.x)}
    return out


def bench_paper_scale(ct, torch, lib):
    """BA-GMRES (B = B_un F) at the paper's data size: 1024 x 1024 x 300
    volume, 180 views of a 1088 x 896 detector (synthetic geometry, see
    synth.workloads.paper_geometry), Poisson data at 1e5 photons.  Full
    30-iteration solve (31 basis vectors), restarted BA-GMRES(10) x 3 cycles
    (11 basis vectors), and the one-shot FDK, each with its image RMSE
    against the attenuation that made the data."""
    import ctypes as C
    from synth import workloads
    from synth.phantoms import rasterize_ellipsoids_torch, poisson_log_counts
    desc = workloads.paper_geometry()
    g = ct.Geometry(desc)
    t0 = time.perf_counter()
    x = rasterize_ellipsoids_torch(workloads.paper_phantom_ellipsoids(), desc.nx, desc.voxel, desc.nz, "cuda")
    ax = ct.ct_project_A(g, x)
    mu = 4.0 / float(ax.max())
    b = torch.from_numpy(poisson_log_counts(703, (ax * mu).double().cpu().numpy().reshape(-1),
                                            1e5).astype(np.float32)).cuda()
    x_ref = x * mu
    del ax
    prep_s = time.perf_counter() - t0

    def rmse(v):
        return float(torch.sqrt(torch.mean((v.double() - x_ref.double()) ** 2)))

    def ws_bytes(solver, iters):
        opts = ct.api.L.SolverOpts(iters, ct.api.L.CT_B_RAMP, ct.api.L.CT_F32, 0.0)
        n = C.c_size_t()
        lib.ct_solver_workspace_bytes(g.handle, solver, C.byref(opts), C.byref(n))
        return n.value

    out = {"workload": "1024x1024x300 volume, 180 views over 360 deg, 1088x896 detector (0.278 mm), "
                       "magnification 2, 12 ellipsoids, Poisson 1e5", "input_generation_s": prep_s}
    ct.ct_ba_gmres(g, b, 2, B="ramp")          # load kernels, size the workspace
    torch.cuda.synchronize()
    lib.ct_profile_reset()
    lib.ct_profile_enable(1)
    t0 = time.perf_counter()
    r = ct.ct_ba_gmres(g, b, ITERS, B="ramp")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lib.ct_profile_enable(0)
    kern = {}
    for name in ("A", "B", "F", "CGS"):
        n_l, t_l = C.c_long(), C.c_double()
        lib.ct_profile_read(name.encode(), C.byref(n_l), C.byref(t_l))
        kern[name] = t_l.value / max(n_l.value, 1)
    # Joseph samples per application of A at this size, counted by the oracle
    n_a = json.load(open(os.path.join(ROOT, "tests", "golden", "update_counts.json")))["paper"]["A_updates"]
    out["full"] = {"iters": r.iters_done, "s": dt, "iters_per_s": r.iters_done / dt,
                   "image_rmse": rmse(r.x), "workspace_GB": ws_bytes(ct.api.L.CT_SOLVER_BA, ITERS) / 1e9,
                   "kernel_ms_per_launch": {"A": kern["A"], "B_un": kern["B"], "F": kern["F"]},
                   "A_samples_per_launch": n_a, "A_samples_per_s": n_a / (kern["A"] * 1e-3)}
    del r
    t0 = time.perf_counter()
    rr = ct.ct_ba_gmres_restarted(g, b, 10, 3, B="ramp")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["restarted_10x3"] = {"iters": rr.iters_done, "s": dt, "iters_per_s": rr.iters_done / dt,
                             "image_rmse": rmse(rr.x),
                             "workspace_GB": ws_bytes(ct.api.L.CT_SOLVER_BA_RESTARTED, 10) / 1e9}
    del rr
    xf = ct.ct_fbp(g, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xf = ct.ct_fbp(g, b, out=xf)
    torch.cuda.synchronize()
    out["FDK"] = {"s": time.perf_counter() - t0, "image_rmse": rmse(xf)}
    del xf
    # the projector's launch settings at this size (the solves above ran
    # with the size heuristic, which is restored afterwards)
    out["projector_setting"] = dict(zip(("view_group", "wg_per_cu"), ct.ct_projector_get_config(g)))
    timed, chosen = ct.ct_tune_projector(g, reps=2)
    ct.ct_projector_config(g, 0, 0)
    out["projector_tuning"] = {"candidates": [{"view_group": v, "wg_per_cu": w, "ms": round(t, 3)}
                                              for v, w, t in timed],
                               "fastest": dict(zip(("view_group", "wg_per_cu"), chosen))}
    return out


def binding_bounds(ceil, g, upd, t_meas, flop_per_upd):
    """The time a kernel cannot beat on this device, from the measured
    ceilings: the largest of its algorithmic HBM bytes (4 n + 4 m) at the
    streaming read rate, its algorithmic FLOP at the FP32 FMA rate and its
    tap bytes (16 per update) at the conflict-free LDS read rate; the tap
    bytes at the rate of the bilinear gather pattern are reported beside."""
    t = {"hbm_ms": 4.0 * (g.n_vox + g.n_rays) / (ceil["hbm_read_gbs"] * 1e9) * 1e3,
         "valu_ms": upd * flop_per_upd / (ceil["fp32_fma_tflops"] * 1e12) * 1e3,
         "lds_peak_ms": upd * 16.0 / (ceil["lds_peak_gbs"] * 1e9) * 1e3}
    bound = max(t.values())
    t["gather_pattern_ms"] = upd * 16.0 / (ceil["lds_gather_gbs"] * 1e9) * 1e3
    t.update({"bound_ms": bound, "measured_ms": t_meas * 1e3, "frac": bound / (t_meas * 1e3)})
    return {k: round(v, 4) for k, v in t.items()}


def kernel_times(ct, lib, g, b, sdt, steps):
    """Average duration of each kernel class over `steps` headline solves,
    from the library's event pairs on the solver's stream (a pass of its
    own, after the timed steps)."""
    import torch
    lib.ct_profile_reset()
    lib.ct_profile_enable(1)
    done = 0
    for _ in range(steps):
        done += ct.ct_ba_gmres(g, b, ITERS, B="ramp", sino_dtype=sdt).iters_done
    torch.cuda.synchronize()
    lib.ct_profile_enable(0)
    kern = {}
    for name in ("A", "B", "F", "CGS"):
        n_l, t_l = ctypes.c_long(), ctypes.c_double()
        lib.ct_profile_read(name.encode(), ctypes.byref(n_l), ctypes.byref(t_l))
        kern[name] = (n_l.value, t_l.value / 1e3)
    return kern, done


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--sino-dtype", default="f32", choices=["f32", "f16"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-siddon", action="store_true")
    ap.add_argument("--no-monitor", action="store_true")
    ap.add_argument("--no-basis16", action="store_true")
    ap.add_argument("--no-fig2", action="store_true")
    ap.add_argument("--paper-scale", action="store_true",
                    help="also solve at the paper's data size (1024x1024x300, 180 x 1088x896)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2201_07408_amd as ct
    from synth import workloads

    torch.cuda.set_device(0)
    desc = workloads.w3_geometry()
    g = ct.Geometry(desc)
    desc2 = workloads.w2_geometry()
    log("bench: generating inputs")
    vol3 = workloads.w3_phantom()
    vol2 = workloads.w2_phantom()
    t_oracle_a3 = None
    if not args.no_cpu:
        log("bench: CPU oracle leg (data from the oracle's projector)")
        clean3, clean2, t_oracle_a3 = oracle_data(desc, vol3, desc2, vol2)
        data_from = "oracle"
    else:
        clean3 = gpu_data(ct, g, torch, vol3)
        clean2 = gpu_data(ct, ct.Geometry(desc2), torch, vol2)
        data_from = "gpu"
    b_host, x_phantom = phantom_scaled_data(vol3, clean3)
    b = torch.from_numpy(b_host).cuda()
    sdt = torch.float16 if args.sino_dtype == "f16" else torch.float32

    log("bench: warmup")
    for _ in range(args.warmup):
        r = ct.ct_ba_gmres(g, b, ITERS, B="ramp", sino_dtype=sdt)
    torch.cuda.synchronize()
    log("bench: timed solves")
    t0 = time.perf_counter()
    done = 0
    step_s = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        # each solve ends by copying its residual history to the host, so the
        # step's wall-clock time is its GPU time plus that copy
        r = ct.ct_ba_gmres(g, b, ITERS, B="ramp", sino_dtype=sdt)
        step_s.append(time.perf_counter() - ts)
        done += r.iters_done
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = done / dt
    x32 = r.x.clone()

    log("bench: kernel timing pass")
    lib = ct.api.L.load()
    kern, done_p = kernel_times(ct, lib, g, b, sdt, args.profile_steps)
    t_a = kern["A"][1] / max(kern["A"][0], 1)
    t_b = kern["B"][1] / max(kern["B"][0], 1)
    t_f = kern["F"][1] / max(kern["F"][0], 1)

    # exact update counts of this geometry, written by the oracle's counter
    # (tests/golden/make_update_counts.py); read as data, the oracle is not run
    counts_path = os.path.join(ROOT, "tests", "golden", "update_counts.json")
    counts = json.load(open(counts_path))["w3"]
    a_upd, b_upd = counts["A_updates"], counts["B_updates"]
    dom = ("A", t_a, a_upd, FLOP_PER_A_UPDATE) if t_a >= t_b else ("B_un", t_b, b_upd, FLOP_PER_B_UPDATE)
    achieved = dom[2] * dom[3] / dom[1]
    traffic = None
    if dom[0] == "A" and projector_src_hash() == A_TRAFFIC_SRC:
        traffic = A_TRAFFIC_BYTES
    line = {
        "metric": "BA-GMRES iters/s at 256^3 cone-beam; A/B voxel-ray updates/s; rel err vs FP64",
        "value": round(value, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "ms_per_step_each": [round(t * 1e3, 3) for t in step_s],
        "ms_per_step_median": round(float(np.median(step_s)) * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if sdt == torch.float32 else "f32 (f16 data storage)",
        "data": "synthetic",
        "config": {"workload": "cone-beam 256^3, 360 views over 360 deg, 384x384 detector, "
                               "ellipsoids + 5% texture, Poisson 1e5 photons, log; BA-GMRES with "
                               "B = ramp-filtered voxel-driven B_un, 30 iterations per step",
                   "iters_per_step": ITERS, "sino_dtype": args.sino_dtype, "data_projector": data_from},
        "A_updates_per_s": a_upd / t_a,
        "B_updates_per_s": b_upd / t_b,
        "kernel_ms_per_launch": {"A": t_a * 1e3, "B_un": t_b * 1e3, "F": t_f * 1e3,
                                 "CGS_per_iteration": kern["CGS"][1] / max(done_p, 1) * 1e3,
                                 "pass": "%d solves after the timed ones, library event pairs" % args.profile_steps},
        "roofline": {"bound": "alu", "kernel": dom[0], "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR, "traffic": traffic},
        # the forward projector's launch setting in the timed solves (the
        # size heuristic; the stored traffic figure was measured with it)
        "projector_setting": dict(zip(("view_group", "wg_per_cu"), ct.ct_projector_get_config(g))),
    }
    # the device's measured ceilings and the bound each projector cannot beat
    log("bench: device ceilings")
    ceil = ct.ct_measure_ceilings()
    line["ceilings"] = {k: round(v, 1) for k, v in ceil.items()}
    line["binding_bound"] = {"A": binding_bounds(ceil, g, a_upd, t_a, FLOP_PER_A_UPDATE),
                             "B_un": binding_bounds(ceil, g, b_upd, t_b, FLOP_PER_B_UPDATE)}
    # the autotuner's view of the same setting: every candidate timed on this
    # geometry, after which the heuristic is restored for the other legs
    log("bench: projector launch settings")
    timed, chosen = ct.ct_tune_projector(g, reps=3)
    ct.ct_projector_config(g, 0, 0)
    line["projector_tuning"] = {"candidates": [{"view_group": v, "wg_per_cu": w, "ms": round(t, 4)}
                                               for v, w, t in timed],
                                "fastest": dict(zip(("view_group", "wg_per_cu"), chosen))}
    if sdt == torch.float32:
        log("bench: FP16 data storage")
        line["fp16_data_storage"] = bench_f16_data(ct, torch, g, b, x_phantom, x32)
        line["fp16_data_storage"]["residual_at_30_fp32_storage"] = r.res[-1]
    # the matched transpose (CGLS with A^T, autograd backward), outside the
    # timed solves: three launches on the same data
    log("bench: matched transpose")
    yat = ct.ct_project_A(g, torch.ones(desc.vol_shape, device=b.device))
    xat = ct.ct_backproject_AT(g, yat)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        xat = ct.ct_backproject_AT(g, yat, out=xat)
    e1.record()
    torch.cuda.synchronize()
    line["AT_ms_per_launch"] = e0.elapsed_time(e1) / 3
    del yat, xat
    if not args.no_fig2:
        log("bench: data-residual curves on the 128^3 workload")
        line["fig2_128cube"] = bench_fig2(ct, torch, clean2, vol2)
    if not args.no_monitor:
        log("bench: monitored solves")
        line["monitor"] = bench_monitor(ct, torch, b, x_phantom, ms_per_step)
    if not args.no_basis16 and sdt == torch.float32:
        log("bench: FP16 Krylov basis")
        line["basis_fp16"] = bench_basis16(ct, torch, lib, g, b, x_phantom, x32)
    if not args.no_siddon:
        log("bench: line-intersection forward model")
        line["siddon_A"] = bench_siddon(ct, torch, lib)
    if args.paper_scale:
        log("bench: paper-size problem")
        line["paper_scale"] = bench_paper_scale(ct, torch, lib)
    if not args.no_batched:
        log("bench: batched 2D slices")
        line["batched_2d"] = bench_batched(ct, torch)
    if not args.no_cpu:
        log("bench: CPU oracle BA-GMRES on the headline workload")
        K = 2
        rk = ct.ct_ba_gmres(g, b, K, B="ramp")
        xk = rk.x.double().cpu().numpy().reshape(-1)
        cb, ref = cpu_baseline(desc, b_host)
        line["cpu_baseline"] = cb
        xr = np.asarray(ref.x).reshape(-1)
        d = np.abs(xk - xr)
        line["rel_err_vs_fp64"] = {
            "x_%d_headline" % K: float(np.linalg.norm(xk - xr) / np.linalg.norm(xr)),
            "x_%d_worst_voxel_of_max" % K: float(d.max() / np.abs(xr).max()),
            "residual_history_%d_worst_entry" % K:
                float(np.max(np.abs(np.array(rk.res) - np.array(ref.res)) / np.array(ref.res))),
            "note": "GPU BA-GMRES(B_FBP) iterate after %d iterations on the full headline workload against the "
                    "FP64 oracle's (same FP32 data)" % K}
        line["rel_err_vs_fp64"].update(sampled_errors(desc, ct, g, torch, x_phantom))
        line["cpu_baseline"]["oracle_projection_s"] = t_oracle_a3
        log("bench: CPU oracle on the 64^2 and 128^3 workloads")
        d1 = workloads.w1_geometry()
        import oracle
        c1 = oracle.project_A(d1, workloads.w1_phantom())
        b1 = (c1 + workloads.relative_gaussian_noise(c1, 0.01, 102)).astype(np.float32).astype(np.float64)
        line["cpu_oracle_configs"] = cpu_small_configs(d1, b1, desc2,
                                                       clean2.astype(np.float32).astype(np.float64))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
