"""Batched sources: one launch over many uneven sources equals per-event
launches bit for bit; HIP-graph replays equal the eager launch; the tuned
launch configuration does not change results."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_14354_amd import workloads as W
from tests.gpu_common import agreement, hist_of_detected, to_records

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def det():
    assert torch.cuda.is_available()
    from paper_2203_14354_amd import runtime
    return runtime.Detector(W.tpc1(), device=0)


def test_batched_equals_per_event_launches(det):
    wl = W.batched_s1(n_events=64)
    src = wl.sources
    out = det.propagate(src, seed=4)["hit_map"].cpu().numpy()
    offs = src.offsets
    for e in range(0, 64, 7):
        one = W.point_sources(src.positions[e:e + 1], counts=[offs[e + 1] - offs[e]])
        row = det.propagate(one, seed=4, pid_base=int(offs[e]))["hit_map"].cpu().numpy()
        assert np.array_equal(row[0], out[e])


def test_event_cache_with_uneven_and_empty_events(det):
    """Per-event maps with prefix offsets are summed per wave in LDS for the
    wave's two most recent events (chunks of 768 ids first).  With events
    of 0 to 20,000 photons (chunks that span many events, rows evicted while
    photons of their events are still in flight) the map equals the
    histogram of the records of the same launch, which adds every detection
    to device memory directly."""
    rng = np.random.default_rng(11)
    n_ev = 600
    counts = rng.choice([0, 1, 7, 100, 1500, 20000], size=n_ev, p=[.1, .1, .2, .3, .2, .1])
    pos = W.uniform_points_in_cylinder(n_ev, W.TPC1_SRC_R, -W.TPC1_SRC_ZHALF, W.TPC1_SRC_ZHALF, 3)
    src = W.point_sources(pos, counts=counts, per_source_events=True)
    cached = det.propagate(src, seed=9)["hit_map"].clone()
    out = det.propagate(src, seed=9, records=True)
    torch.cuda.synchronize()
    assert torch.equal(cached, out["hit_map"])
    rec = to_records(out["records"])
    assert np.array_equal(cached.cpu().numpy(), hist_of_detected(rec, n_ev, det.n_channels))
    assert np.all(cached.cpu().numpy()[counts == 0] == 0)  # empty events get no hits


@pytest.mark.parametrize("counts", [[0, 5, 1, 0, 9, 0], [0] + [100] * 7 + [0],
                                    [0] + [95] * 9 + [0], [3, 0, 4000, 0, 2]],
                         ids=["15-photons", "700-photons", "855-photons", "4005-photons"])
def test_event_cache_at_the_big_chunk_boundary(det, counts):
    """Per-event launches with no, exactly one or a few chunks of 768 ids in
    the event-cache launch's first part (0.9 n / 768, rounded down: 0, 0, 1
    and 4 here) and empty events at both ends: the map equals that of the
    records launch and the histogram of its records."""
    counts = np.asarray(counts)
    pos = W.uniform_points_in_cylinder(len(counts), W.TPC1_SRC_R, -W.TPC1_SRC_ZHALF,
                                       W.TPC1_SRC_ZHALF, 5)
    src = W.point_sources(pos, counts=counts, per_source_events=True)
    cached = det.propagate(src, seed=21)["hit_map"].clone()
    out = det.propagate(src, seed=21, records=True)
    torch.cuda.synchronize()
    assert torch.equal(cached, out["hit_map"])
    rec = to_records(out["records"])
    assert len(rec) == counts.sum()
    assert np.array_equal(cached.cpu().numpy(), hist_of_detected(rec, len(counts), det.n_channels))
    assert np.all(cached.cpu().numpy()[counts == 0] == 0)
    if counts.sum() > 100:
        assert int(cached.sum()) > 0


def test_batched_records_match_oracle(det):
    wl = W.batched_s1(n_events=16)
    src = wl.sources
    res = det.propagate(src, seed=8, records=True)
    torch.cuda.synchronize()
    gpu = to_records(res["records"])
    ref = oracle.run(oracle.Scene(W.tpc1()), src, seed=8)
    assert np.array_equal(gpu["event"], ref["records"]["event"])
    assert agreement(gpu, ref["records"]).mean() >= 0.999
    hm = res["hit_map"].cpu().numpy()
    assert hm.shape == (16, 38)
    assert np.abs(hm - ref["hit_map"]).sum() <= 2 * (~agreement(gpu, ref["records"])).sum()


def test_graph_replay_equals_eager(det):
    from paper_2203_14354_amd.batched import BatchedRunner
    wl = W.batched_s1(n_events=512)
    eager = det.propagate(wl.sources, seed=6)["hit_map"].clone()
    r = BatchedRunner(det, wl.sources, seed=6, autotune=True, use_graph=True,
                      tune_photons=500_000)
    for k in range(3):
        got = r.run().clone()
        torch.cuda.synchronize()
        assert torch.equal(got, eager), k
        # eager work and a synchronization between replays
        other = det.propagate(W.small_tpc(photons_per_point=1000).sources, seed=k)["hit_map"]
        torch.cuda.synchronize()
        assert int(other.sum()) > 0


def test_captured_launch_keeps_its_own_work_counter(det):
    """A launch captured in a graph keeps its work counter for every replay.
    70 eager launches of the same context (more than its ring of 64 eager
    counters) run on another stream while the graph replays, each launch at
    one workgroup per CU so that they share the GPU: no eager launch may take
    the replay's counter (split or repeated photons would change the maps)."""
    one = dict(blocks_per_cu=1)
    big = det.sources(W.small_tpc(photons_per_point=200_000).sources)
    small = det.sources(W.small_tpc(photons_per_point=2_000).sources)
    ref_big = det.propagate(big, seed=21, launch=one)["hit_map"].clone()
    ref_small = det.propagate(small, seed=22, launch=one)["hit_map"].clone()
    hm = torch.zeros_like(ref_big)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        hm.zero_()
        det.propagate(big, seed=21, hit_map=hm, launch=one)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hm.zero_()
        det.propagate(big, seed=21, hit_map=hm, launch=one)
    torch.cuda.synchronize()
    for k in range(3):
        maps = [torch.zeros_like(ref_small) for _ in range(70)]
        torch.cuda.synchronize()
        side.wait_stream(torch.cuda.current_stream())
        g.replay()
        with torch.cuda.stream(side):
            for m in maps:
                det.propagate(small, seed=22, hit_map=m, launch=one)
        torch.cuda.synchronize()
        assert torch.equal(hm, ref_big), k
        for m in maps:
            assert torch.equal(m, ref_small), k


def test_autotuned_config_gives_identical_results(det):
    wl = W.batched_s1(n_events=256)
    a = det.propagate(wl.sources, seed=1)["hit_map"].clone()
    cfg = det.autotune(wl.sources, sample_photons=300_000)
    assert cfg["block_size"] in (64, 128, 256)
    b = det.propagate(wl.sources, seed=1, launch=cfg)["hit_map"]
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_lce_map_batch_invariance_and_oracle():
    from paper_2203_14354_amd import lcemap
    det = lcemap.tpc1_lce_map_detector()
    cen = W.equal_volume_cell_centroids(6, 6, 6, W.TPC1_SRC_R, -W.TPC1_SRC_ZHALF,
                                        W.TPC1_SRC_ZHALF)
    h1, g1 = lcemap.lce_map(det, cen, 500, seed=3, batch_cells=216)
    h2, g2 = lcemap.lce_map(det, cen, 500, seed=3, batch_cells=50)
    torch.cuda.synchronize()
    assert torch.equal(h1, h2)
    assert torch.allclose(g1, g2, rtol=1e-9, atol=1e-9)
    mesh = W.tpc1(plane=True)
    sc = oracle.Scene(mesh, channel_of_sensor=W.tpc1_top_bottom_channels(mesh), n_channels=2)
    h = h1.cpu().numpy()
    for c in (0, 77, 215):
        src = W.point_sources(cen[c:c + 1], count_per_source=500, per_source_events=True)
        ref = oracle.run(sc, src, seed=3, pid_base=c * 500)["hit_map"][0]
        assert np.abs(ref - h[c]).max() <= 1, (c, ref, h[c])
