"""Full-size parity of the batched, differentiable and light-collection-map
workloads, in the launch configurations the benchmark times.

For each: the full launch runs as the benchmark runs it; launches that also
write per-photon records (over the whole workload, or over sampled parts of
it with the same photon ids) give the same integer tallies, and the oracle
recomputes at least 20,000 photons sampled over the whole id range (bar:
99.9 % same terminal flag, final triangle, sensor and step count).  Gradient tallies equal the sums of the records'
per-photon scores (FP64, up to summation order), and the scores of agreeing
photons equal the oracle's within FP32 rounding.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_14354_amd import workloads as W
from tests.gpu_common import agreement, detected_scores, hist_of_detected, to_records

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available()
    from paper_2203_14354_amd import runtime
    return runtime


RUN = 500  # consecutive photon ids per sampled run


def _sample_runs(n, n_runs, seed):
    """Launch-local ids of n_runs runs of RUN consecutive photons spread over [0, n)."""
    starts = np.sort(np.random.default_rng(seed).choice(n // RUN, n_runs, replace=False)) * RUN
    return starts, (starts[:, None] + np.arange(RUN)[None, :]).ravel()


def _oracle_runs(sc, src, seed, starts, grad=False, pid_base=0):
    """Oracle records of the runs of RUN photons beginning at the given ids."""
    return np.concatenate([oracle.run(sc, src, seed=seed, pid_base=pid_base, i_begin=int(s),
                                      i_end=int(s) + RUN, grad=grad, hit_map=False)["records"]
                           for s in starts])


def test_batched_s1_full_size_sampled(rt):
    """4,096 log-normal sources (about 2.4e7 photons), per-event hit maps, the
    benchmark's eager launch: the launch with records gives the same map, the
    map is the histogram of the records, and 20,000 sampled photons agree with
    the oracle."""
    wl = W.batched_s1()
    det = rt.Detector(wl.mesh, device=0)
    src = wl.sources
    n = src.n_photons
    assert n > 2e7 and src.n_events == 4096
    plain = det.propagate(src, seed=2)["hit_map"].clone()
    out = det.propagate(src, seed=2, records=True)
    torch.cuda.synchronize()
    assert torch.equal(plain, out["hit_map"])
    rec = to_records(out["records"])
    del out
    assert np.array_equal(plain.cpu().numpy(), hist_of_detected(rec, 4096, det.n_channels))
    assert np.array_equal(np.bincount(rec["event"], minlength=4096), np.diff(src.offsets))
    starts, ids = _sample_runs(n, 40, 2)
    o = _oracle_runs(oracle.Scene(wl.mesh), src, 2, starts)
    g = rec[ids]
    assert np.array_equal(g["event"], o["event"])
    assert len(g) == 20_000 and agreement(g, o).mean() >= 0.999


def test_differentiable_full_size_sampled(rt):
    """1e7 photons with fused FP64 gradient tallies (the benchmark's launch:
    38 channels, so the tallies are summed per workgroup in LDS): the hit map
    equals that of the launch with records, the Jacobian equals the records'
    per-sensor score sums, and 20,000 sampled photons agree with the oracle,
    their scores within FP32 rounding."""
    wl = W.differentiable(photons_per_point=1_000_000)
    det = rt.Detector(wl.mesh, device=0)
    src = wl.sources
    n = src.n_photons
    assert n == 10_000_000
    fused = det.propagate(src, seed=1, grad=True)
    # records carry the score inputs only when the launch tallies gradients
    # (device-memory atomics: launches with records never use the LDS tallies)
    out = det.propagate(src, seed=1, grad=True, records=True)
    torch.cuda.synchronize()
    assert torch.equal(fused["hit_map"], out["hit_map"])
    rec = to_records(out["records"])
    G, Gd = fused["grad"].cpu().numpy()[0], out["grad"].cpu().numpy()[0]
    del out
    s = detected_scores(rec, wl.mesh.materials)
    detm = (rec["flag"] & 0xFF) == oracle.F_DETECT
    ref = np.zeros_like(G)
    np.add.at(ref, rec["sensor"][detm], s[detm])
    assert np.abs(ref).min() > 0
    assert np.allclose(G, ref, rtol=1e-9, atol=1e-6)
    assert np.allclose(G, Gd, rtol=1e-9, atol=1e-6)
    starts, ids = _sample_runs(n, 40, 3)
    o = _oracle_runs(oracle.Scene(wl.mesh), src, 1, starts, grad=True)
    g = rec[ids]
    ag = agreement(g, o)
    assert len(g) == 20_000 and ag.mean() >= 0.999
    m = ag & ((g["flag"] & 0xFF) == oracle.F_DETECT)
    assert m.sum() > 2000
    sg, so = detected_scores(g, wl.mesh.materials), detected_scores(o, wl.mesh.materials)
    assert np.allclose(sg[m], so[m], rtol=1e-3, atol=1e-3)
    assert np.array_equal(g["n_scatter"][m], o["n_scatter"][m])


def test_lce_map_full_size_sampled(rt):
    """64^3 cells x 1e4 photons (2.6e9 photons) in the benchmark's batches of
    16,384 cells: six sampled cells rerun on their own with records give the
    same {top, bottom} counts and gradients, and all 10,000 photons of each
    agree with the oracle (60,000 photons)."""
    from paper_2203_14354_amd import lcemap
    det = lcemap.tpc1_lce_map_detector()
    cen = W.equal_volume_cell_centroids(64, 64, 64, W.TPC1_SRC_R, -W.TPC1_SRC_ZHALF,
                                        W.TPC1_SRC_ZHALF)
    hits, g = lcemap.lce_map(det, cen, 10_000, seed=4, batch_cells=16384)
    torch.cuda.synchronize()
    hits, g = hits.cpu().numpy(), g.cpu().numpy()
    assert hits.shape == (64 ** 3, 2) and g.shape == (64 ** 3, 2, 4)
    lce = hits.sum(axis=1) / 10_000
    assert 0.1 < lce.min() and lce.max() < 0.4
    mesh = W.tpc1(plane=True)
    sc = oracle.Scene(mesh, channel_of_sensor=W.tpc1_top_bottom_channels(mesh), n_channels=2)
    agrees = []
    for c in (0, 16383, 16384, 131071, 200000, 64 ** 3 - 1):
        one = W.point_sources(cen[c:c + 1], count_per_source=10_000, per_source_events=True)
        out = det.propagate(one, seed=4, pid_base=c * 10_000, grad=True, records=True)
        torch.cuda.synchronize()
        assert np.array_equal(out["hit_map"].cpu().numpy()[0], hits[c])
        assert np.allclose(out["grad"].cpu().numpy()[0], g[c], rtol=1e-9, atol=1e-9)
        rec = to_records(out["records"])
        o = oracle.run(sc, one, seed=4, pid_base=c * 10_000, hit_map=False)["records"]
        agrees.append(agreement(rec, o))
    ag = np.concatenate(agrees)
    assert len(ag) == 60_000 and ag.mean() >= 0.999
