"""Gradient tallies on the GPU: per-photon scores against the oracle, the
backward replay against the contraction of the fused Jacobian, the analytic
sphere, and common-random-number finite differences at the base point and the
ends of the paper's systematic ranges."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2203_14354_amd import workloads as W
from tests.gpu_common import agreement, detected_scores as _scores, to_records
from tests.helpers import face_average

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available()
    from paper_2203_14354_amd import runtime
    return runtime


def test_fused_tallies_match_records_and_oracle(rt):
    wl = W.differentiable(n_points=3, photons_per_point=20_000)
    det = rt.Detector(wl.mesh, device=0)
    out = det.propagate(wl.sources, seed=7, grad=True, records=True)
    torch.cuda.synchronize()
    gpu = to_records(out["records"])
    G = out["grad"].cpu().numpy()[0]
    s = _scores(gpu, wl.mesh.materials)
    # the tallies are the per-sensor sums of the per-photon scores (FP64 atomics)
    detm = (gpu["flag"] & 0xFF) == 1
    ref = np.zeros_like(G)
    np.add.at(ref, gpu["sensor"][detm], s[detm])
    assert np.allclose(G, ref, rtol=1e-9, atol=1e-9)
    # per-photon scores of agreeing photons equal the oracle's (FP32 vs FP64)
    orc = oracle.run(oracle.Scene(wl.mesh), wl.sources, seed=7, grad=True)
    o = orc["records"]
    ag = agreement(gpu, o)
    assert ag.mean() >= 0.999
    so = _scores(o, wl.mesh.materials)
    m = ag & detm
    assert np.allclose(s[m], so[m], rtol=1e-3, atol=1e-3)
    assert np.array_equal(gpu["n_scatter"][m], o["n_scatter"][m])
    # and the tallied Jacobian agrees with the oracle's within the disagreeing photons
    diff = np.abs(G - orc["grad"][0]).sum(axis=0)
    bound = np.abs(s[~ag]).sum(axis=0) + np.abs(so[~ag]).sum(axis=0) + 1e-3 * np.abs(G).sum(0)
    assert np.all(diff <= bound + 1e-6)


def test_backward_replay_equals_fused_contraction(rt):
    wl = W.differentiable(n_points=4, photons_per_point=50_000)
    det = rt.Detector(wl.mesh, device=0)
    out = det.propagate(wl.sources, seed=3, grad=True)
    g_out = torch.linspace(-1.0, 2.0, det.n_channels, device="cuda").reshape(1, -1)
    gp = det.backward(wl.sources, g_out, seed=3)
    torch.cuda.synchronize()
    G = out["grad"].double()
    expect = torch.einsum("ec,ecp->p", g_out.double(), G)
    assert torch.allclose(gp, expect, rtol=1e-6, atol=1e-6)


def test_autograd_function_both_modes(rt):
    from paper_2203_14354_amd.autograd import base_params, hits
    wl = W.differentiable(n_points=2, photons_per_point=50_000)
    det = rt.Detector(wl.mesh, device=0)
    p = base_params(wl.mesh).requires_grad_(True)
    w = torch.arange(det.n_channels, dtype=torch.float64, device="cuda").reshape(1, -1)
    grads = []
    for mode in ("fused", "replay"):
        h = hits(p, det, wl.sources, seed=5, mode=mode)
        (h * w).sum().backward()
        grads.append(p.grad.clone())
        p.grad = None
    assert torch.allclose(grads[0], grads[1], rtol=1e-6, atol=1e-6)
    assert torch.all(torch.isfinite(grads[0]))


def test_sphere_absorption_gradient_analytic(rt):
    lam = 0.1
    m = W.sphere(0.1, level=5, lam_abs=lam)
    det = rt.Detector(m, device=0)
    n = 2_000_000
    out = det.propagate(W.point_sources([[0, 0, 0]], count_per_source=n), seed=2, grad=True,
                        records=True)
    torch.cuda.synchronize()
    g = out["grad"].cpu().numpy()[0, 0] / n
    P = out["hit_map"].sum().item() / n
    expP = face_average(m.vertices, m.triangles, [0, 0, 0], lambda d: np.exp(-d / lam))
    expG = face_average(m.vertices, m.triangles, [0, 0, 0], lambda d: d / lam ** 2 * np.exp(-d / lam))
    assert abs(P - expP) < 4 * math.sqrt(expP * (1 - expP) / n)
    rec = to_records(out["records"])
    sc = np.where((rec["flag"] & 0xFF) == 1, rec["path_len"] / lam ** 2, 0.0)
    assert abs(g[0] - expG) < 4 * sc.std() / math.sqrt(n)


def _batched_estimates(det, src, params, seed, n_batches, per_batch, gm=0):
    """Per-batch total hits and per-batch score tallies at the given parameters."""
    from paper_2203_14354_amd.autograd import apply_params
    apply_params(det, params, gm)
    H, G = [], []
    for b in range(n_batches):
        out = det.propagate(src, seed=seed, pid_base=b * per_batch, n_photons=per_batch, grad=True)
        H.append(out["hit_map"].sum())
        G.append(out["grad"].sum(dim=(0, 1)))
    torch.cuda.synchronize()
    return torch.stack(H).double().cpu().numpy(), torch.stack(G).cpu().numpy()


# (parameter, values moved off the base point): the base point (L_abs 50 m,
# L_R 0.4 m, R 0.95, T 0.9) for all four parameters, and the ends of the
# systematic ranges of table tab:lce_sys for the first three
FD_CASES = [(0, {}), (1, {}), (2, {}), (3, {}),
            (0, {0: 10.0}), (0, {0: 100.0}), (1, {1: 0.3}), (1, {1: 0.6}),
            (2, {2: 0.90}), (2, {2: 0.99})]


def test_crn_finite_differences(rt):
    """d(total hits)/d theta_p: the score-function tallies against central
    finite differences with common random numbers (same seed and photon ids;
    steps of 2 % for the lengths, 0.005 for R and T), at the base point and at
    the range ends.  Error bars from 50 batch means of 2e5 photons, the two
    estimates' variances added (their positive correlation makes this
    conservative); the pulls must have chi^2/ndf < 1.5 and none may exceed 4."""
    from paper_2203_14354_amd.autograd import base_params
    nb, per = 50, 200_000
    wl = W.differentiable(n_points=1, photons_per_point=nb * per)
    det = rt.Detector(wl.mesh, device=0)
    ds = det.sources(wl.sources)
    base = base_params(wl.mesh).numpy()
    pulls = []
    for p, moved in FD_CASES:
        x0 = base.copy()
        for k, v in moved.items():
            x0[k] = v
        h = 0.02 * x0[p] if p < 2 else 0.005
        _, G = _batched_estimates(det, ds, x0, 11, nb, per)
        lo, hi = x0.copy(), x0.copy()
        lo[p] -= h
        hi[p] += h
        Hl, _ = _batched_estimates(det, ds, lo, 11, nb, per)
        Hh, _ = _batched_estimates(det, ds, hi, 11, nb, per)
        fd = (Hh - Hl) / (2 * h)
        sc = G[:, p]
        se = math.sqrt(fd.var(ddof=1) / nb + sc.var(ddof=1) / nb)
        pulls.append((fd.mean() - sc.mean()) / se)
        print(f"param {p} at {x0.tolist()}: FD {fd.mean():.6g}, score {sc.mean():.6g}, "
              f"se {se:.3g}, pull {pulls[-1]:+.2f}")
    pulls = np.array(pulls)
    assert np.abs(pulls).max() < 4.0, pulls
    assert (pulls ** 2).mean() < 1.5, pulls


def test_block_tallies_equal_global_tallies(rt):
    """A launch with few hit-map cells can sum its hits and gradient scores per
    workgroup in LDS and add them to global memory once per workgroup
    (block_tally = 1), or add every detection to global memory directly
    (block_tally = -1).  Both follow the same photons: hits identical,
    gradients equal up to summation order.  With one event per source (300 x
    38 cells, too many for LDS) the tallies always go to global memory, and
    summed over the sources they equal the single-event tallies."""
    wl = W.differentiable(n_points=300, photons_per_point=2_000)
    det = rt.Detector(wl.mesh, device=0)
    per = dataclasses.replace(wl.sources, per_source_events=True)
    for grad in (False, True):
        a = det.propagate(wl.sources, seed=5, grad=grad, launch={"block_tally": 1})
        c = det.propagate(wl.sources, seed=5, grad=grad, launch={"block_tally": -1})
        b = det.propagate(per, seed=5, grad=grad, launch={"block_tally": 1})
        torch.cuda.synchronize()
        assert a["hit_map"].shape == (1, det.n_channels) and b["hit_map"].shape == (300, det.n_channels)
        assert torch.equal(a["hit_map"], c["hit_map"])
        assert torch.equal(a["hit_map"][0], b["hit_map"].sum(dim=0))
        assert int(a["hit_map"].sum()) > 100_000
        if grad:
            ga = a["grad"][0].cpu().numpy()
            for other in (c["grad"][0], b["grad"].sum(dim=0)):
                assert np.allclose(ga, other.cpu().numpy(), rtol=1e-10, atol=1e-12 * np.abs(ga).max())


def test_block_tally_config_is_validated(rt):
    from paper_2203_14354_amd._lib import XpError
    wl = W.differentiable(n_points=2, photons_per_point=100)
    det = rt.Detector(wl.mesh, device=0)
    with pytest.raises(XpError):
        det.propagate(wl.sources, seed=0, launch={"block_tally": 2})
    cfg = det.autotune(wl.sources, sample_photons=50_000)
    assert cfg["block_tally"] in (0, 1)  # never turned off by a hit-map timing


def test_block_tallies_with_several_events(rt):
    """Per-source events whose tallies fit LDS beside the traversal stacks
    (10 events x 38 channels of hits; 2 events with FP64 scores; a 4-event
    time histogram of 512 bins): summed per workgroup (block_tally 1) they
    equal the device-memory tallies (block_tally -1), hits and times exactly,
    gradients up to summation order."""
    wl = W.differentiable(n_points=10, photons_per_point=30_000)
    det = rt.Detector(wl.mesh, device=0)
    ten = dataclasses.replace(wl.sources, per_source_events=True)
    two = W.point_sources(wl.sources.positions[:2], count_per_source=100_000, per_source_events=True)
    four = W.point_sources(wl.sources.positions[:4], count_per_source=30_000, per_source_events=True)
    res = {}
    for bt in (1, -1):
        L = {"block_tally": bt}
        res[bt] = (det.propagate(ten, seed=9, launch=L)["hit_map"],
                   det.propagate(two, seed=9, grad=True, launch=L),
                   det.propagate(four, seed=3, time_hist=512, time_bin_ns=0.25, launch=L))
    torch.cuda.synchronize()
    hm = res[1][0]
    assert hm.shape == (10, det.n_channels) and torch.equal(hm, res[-1][0])
    assert np.all(hm.sum(dim=1).cpu().numpy() > 1000)  # every event got its own photons
    a, b = res[1][1], res[-1][1]
    assert a["hit_map"].shape == (2, det.n_channels) and torch.equal(a["hit_map"], b["hit_map"])
    ga, gb = a["grad"].cpu().numpy(), b["grad"].cpu().numpy()
    assert np.allclose(ga, gb, rtol=1e-10, atol=1e-12 * np.abs(gb).max())
    ta, tb = res[1][2]["time_hist"], res[-1][2]["time_hist"]
    assert ta.shape == (4, 512) and torch.equal(ta, tb) and int(ta.sum()) > 4000
    assert torch.equal(res[1][2]["hit_map"], res[-1][2]["hit_map"])
