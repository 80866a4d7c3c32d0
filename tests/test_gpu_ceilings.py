"""The measured device ceilings (HBM streaming, FP32 issue rates, bilinear
samples from LDS and from L2) that the kernels' rooflines are read
against: finite, within the physical range of one MI355X, and ordered as
the hardware orders them."""
import math

import pytest

import paper_2201_07408_amd as ct

from gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_ceilings_are_plausible():
    say("device ceilings")
    c = ct.ct_measure_ceilings()
    say(c)
    assert all(math.isfinite(v) and v > 0.0 for v in c.values())
    # HBM3E peak 8 TB/s: streaming rates below it and above a tenth of it
    assert 800.0 < c["hbm_copy_gbs"] < 8000.0
    assert 800.0 < c["hbm_read_gbs"] < 8000.0
    # FP32 vector: below the 157.3 TFLOP/s of the packed peak
    assert 5.0 < c["fp32_fma_tflops"] <= 160.0
    assert 5.0 < c["fp32_add_tflops"] <= 160.0
    # taps from LDS come faster than taps gathered through the caches
    assert c["lds_bilinear_gsps"] > c["l2_bilinear_gsps"] > 0.0
    # the taps alone: LDS (at most 256 bytes per clock with 16-byte reads on
    # each of 256 CUs at 2.4 GHz, 157.3 TB/s) above L2
    assert 1000.0 < c["lds_gather_gbs"] <= 157300.0
    assert c["lds_gather_gbs"] > c["l2_gather_gbs"] > 0.0
    # conflict-free reads reach more of the LDS than the gather pattern
    assert c["lds_gather_gbs"] < c["lds_peak_gbs"] <= 157300.0
