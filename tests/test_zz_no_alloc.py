"""The allocation-free forward entry point (xp_propagate_static, through the
C ABI) against xp_propagate: identical integer hit maps, photon records and
counters, on two calls in a row, the second with fewer photons (the fixed
device scratch keeps the first call's work counter and stack entries)."""
import numpy as np
import pytest
import torch

from paper_2203_14354_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_14354_amd import runtime
    return runtime


def _compare(det, ds, n, seed, with_records):
    ref = det.propagate(ds, seed=seed, n_photons=n, records=with_records, stats=with_records)
    hm = torch.zeros_like(ref["hit_map"])
    rec = torch.empty_like(ref["records"]) if with_records else None
    st = torch.zeros_like(ref["stats"]) if with_records else None
    det.propagate_static(ds, hm, seed=seed, n_photons=n, records=rec, stats=st)
    torch.cuda.synchronize()
    assert int(hm.sum()) > 0
    assert torch.equal(hm, ref["hit_map"])
    if with_records:
        assert torch.equal(rec, ref["records"])
        # terminal flags, geometry errors, steps, nodes, triangles, lane slots
        assert torch.equal(st[:14], ref["stats"][:14])


def test_static_entry_point_small_tpc(rt):
    det = rt.Detector(W.tpc1(), device=0)
    ds = det.sources(W.small_tpc().sources)
    _compare(det, ds, 100_000, 3, True)
    _compare(det, ds, 30_011, 4, True)


def test_static_entry_point_darwin(rt):
    """The DARWIN-scale BVH needs 57 stack entries per lane: at the default five
    workgroups per CU the overflow area would exceed the 64 MiB scratch, so the
    call runs four; the hit maps must not change."""
    det = rt.Detector(W.darwin(), device=0)
    assert det.bvh["max_stack"] * 4 * 256 * 256 * 5 > 64 << 20
    ds = det.sources(W.darwin_tpc(n_photons=1_000_000, mesh=det.mesh).sources)
    _compare(det, ds, 1_000_000, 5, False)
    _compare(det, ds, 200_003, 6, True)


def test_static_entry_point_per_event_maps(rt):
    """Per-event maps with prefix offsets take the event-cache path (chunks of
    768 ids first, rows summed per wave in LDS) with the work counter in
    the fixed scratch: the maps equal xp_propagate's, twice in a row, the
    second launch smaller."""
    det = rt.Detector(W.tpc1(), device=0)
    for n_ev, seed in ((200, 11), (37, 12)):
        ds = det.sources(W.batched_s1(n_events=n_ev).sources)
        ref = det.propagate(ds, seed=seed)["hit_map"]
        hm = torch.zeros_like(ref)
        det.propagate_static(ds, hm, seed=seed)
        torch.cuda.synchronize()
        assert hm.shape == (n_ev, det.n_channels) and int(hm.sum()) > 0
        assert torch.equal(hm, ref)


def test_static_entry_point_rejects_a_launch_that_does_not_fit(rt):
    from paper_2203_14354_amd._lib import XpError
    det = rt.Detector(W.darwin(), device=0)
    ds = det.sources(W.darwin_tpc(n_photons=10_000, mesh=det.mesh).sources)
    hm = torch.zeros((1, det.n_channels), dtype=torch.int32, device="cuda")
    with pytest.raises(XpError, match="scratch"):
        det.propagate_static(ds, hm, seed=1, launch=dict(blocks_per_cu=5))
    torch.cuda.synchronize()
    assert int(hm.sum()) == 0
