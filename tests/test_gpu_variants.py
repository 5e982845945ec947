"""GPU parity on the paper's design variants (section "Alternative designs"):
the same kernels on reflective electrodes, a single-phase TPC, no bottom
array and the 4-pi side arrays of 6,480 PMTs or 87,120 SiPMs.

Bars, on every photon of a 200,000-photon launch against the oracle: the same
terminal flag, final triangle, sensor and step count for >= 99.9 % of them;
the {top, bottom, side} hit maps within chi^2/ndf < 1.2 of the oracle's; the
hit map identical to the histogram of the GPU's own photon records.

The variant without the bottom array keeps photons longest (42 steps against
30, most of them reflections off the 0.99 PTFE floor, a fan of 256 wedges
whose shared edges the FP32 and FP64 searches resolve differently within
rounding of the edge).  There the oracle's own FP32 build departs from its
FP64 build on 0.17 % of the photons, and the bar is that rate: the GPU may
depart from the FP64 oracle no more often than single-precision arithmetic
itself does (within 4 standard errors).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2203_14354_amd import workloads as W
from tests.gpu_common import agreement, chi2_ndf, hist_of_detected, to_records

pytestmark = pytest.mark.gpu

VARIANTS = [dict(coating="all"), dict(coating="gate"), dict(single_phase=True),
            dict(bottom_array=False), dict(side_array="pmt2"), dict(side_array="pmt2", fsr=None),
            dict(side_array="sipm", fsr="coated")]
FP32_BAR = ({"bottom_array": False},)


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_14354_amd import runtime
    return runtime


@pytest.mark.parametrize("kw", VARIANTS, ids=lambda kw: "-".join(f"{k}={v}" for k, v in kw.items()))
def test_variant_matches_oracle(rt, kw):
    mesh = W.darwin(**kw)
    ch = W.darwin_array_channels(mesh)
    det = rt.Detector(mesh, device=0, channel_of_sensor=ch, n_channels=3)
    n = 200_000
    src = W.darwin_tpc(n_photons=n, mesh=mesh).sources
    out = det.propagate(src, seed=12, records=True)
    torch.cuda.synchronize()
    g = to_records(out["records"])
    hm = out["hit_map"].cpu().numpy()
    assert np.array_equal(hm, hist_of_detected(g, 1, 3, channel=ch))
    assert not np.any(g["flag"] & oracle.F_GEOMETRY_ERROR)
    ref = oracle.run(oracle.Scene(mesh, channel_of_sensor=ch, n_channels=3, use_bvh=True), src,
                     seed=12)
    ag = agreement(g, ref["records"])
    assert chi2_ndf(hm, ref["hit_map"]) < 1.2
    assert np.array_equal(hist_of_detected(g[ag], 1, 3, channel=ch),
                          hist_of_detected(ref["records"][ag], 1, 3, channel=ch))
    if kw not in FP32_BAR:
        assert ag.mean() >= 0.999, ag.mean()
        return
    r32 = oracle.run(oracle.Scene(mesh, channel_of_sensor=ch, n_channels=3, use_bvh=True,
                                  fp32=True), src, seed=12, hit_map=False)["records"]
    a32 = agreement(r32, ref["records"]).mean()
    se = math.sqrt(a32 * (1 - a32) / n)
    assert ag.mean() >= a32 - 4 * se, (ag.mean(), a32)
