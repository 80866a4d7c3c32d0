"""Operators at the paper's data size (1024 x 1024 x 300 volume, 180 views
of a 1088 x 896 detector): sampled rays and voxels against the oracle, and
the ramp filter on rows of 1088 bins."""

import dataclasses

import numpy as np
import pytest
import torch

import oracle
import paper_2201_07408_amd as ct
from synth import workloads
from tests.gpu_helpers import assert_close, special_rays, dev, f32, host, rel, say

pytestmark = pytest.mark.gpu


def test_paper_size_A_and_Bun_sampled():
    desc = workloads.paper_geometry()
    g = ct.Geometry(desc)
    say("paper size: volume")
    gen = torch.Generator(device="cuda").manual_seed(77)
    x = torch.rand(desc.vol_shape, device="cuda", generator=gen)
    y = ct.ct_project_A(g, x)
    xh = x.double().cpu().numpy()
    rng = np.random.default_rng(78)
    rays = np.union1d(rng.choice(desc.n_rays, size=600, replace=False), special_rays(desc, rows=[0, 15, 16, desc.nv - 1]))
    say("paper size: oracle rays")
    ref = oracle.project_A_rays(desc, xh, rays)
    got = y.reshape(-1)[torch.from_numpy(rays).cuda()].double().cpu().numpy()
    assert_close(got, ref, 1e-5, "paper size A sampled rays")
    del x, xh
    q = torch.rand(desc.sino_shape, device="cuda", generator=gen)
    xb = ct.ct_backproject_B(g, q).reshape(-1)
    vox = rng.choice(desc.n_vox, size=600, replace=False)
    say("paper size: oracle voxels")
    refb = oracle.backproject_Bun_voxels(desc, q.double().cpu().numpy(), vox)
    assert_close(xb[torch.from_numpy(vox).cuda()].double().cpu().numpy(), refb, 1e-5, "paper size B_un sampled voxels")


def test_ramp_rows_of_1088_bins():
    desc = dataclasses.replace(workloads.paper_geometry(), n_views=2, nz=8, nv=40)
    g = ct.Geometry(desc)
    q = f32(np.random.default_rng(79).normal(size=desc.sino_shape))
    assert_close(host(ct.ct_ramp_filter(g, dev(q))), oracle.ramp(desc, q), 1e-5, "F 1088 bins")
