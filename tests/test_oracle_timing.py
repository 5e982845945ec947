"""Pins of the oracle's arrival-time and photon-loss tallies.

The scintillation time profile (section "Optical properties": singlet and
triplet decay constants and the singlet fraction) is checked against its
distribution; times of flight against closed forms (path length times n / c);
the t90 quantile rule against hand-computed histograms and against the
analytic quantile of the decay profile; the loss table (section "Sources of
photon losses") against a closed-form absorption probability and against the
partition of the photons by terminal flag.  None of these tests needs a GPU.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import optimize, stats

from paper_2203_14354_amd import workloads as W
from tests.helpers import binom_sigma

C_M_PER_NS = 0.299792458
TAU1, TAU3, FS = W.SCINT_TAU_SINGLET_NS, W.SCINT_TAU_TRIPLET_NS, W.SINGLET_FRACTION_NR


def mixture_cdf(t, fs=FS, t1=TAU1, t3=TAU3):
    return fs * (1.0 - np.exp(-t / t1)) + (1.0 - fs) * (1.0 - np.exp(-t / t3))


def test_emission_time_distribution(oracle_lib):
    n = 200_000
    t, singlet = oracle_lib.emission_time(seed=3, pid0=0, n=n, tau_singlet=TAU1,
                                          tau_triplet=TAU3, singlet_fraction=FS)
    assert np.all(t > 0) and np.all(np.isfinite(t))
    k = singlet.sum()
    assert abs(k / n - FS) < 5 * binom_sigma(FS, n)
    # each state decays exponentially with its own constant
    for sel, tau in ((singlet == 1, TAU1), (singlet == 0, TAU3)):
        assert stats.kstest(t[sel], "expon", args=(0, tau)).pvalue > 1e-3
        assert abs(t[sel].mean() - tau) < 5 * tau / math.sqrt(sel.sum())
    # and the whole sample follows the two-component profile
    assert stats.kstest(t, mixture_cdf).pvalue > 1e-3


def test_emission_time_pure_states(oracle_lib):
    t1, s1 = oracle_lib.emission_time(1, 0, 50_000, TAU1, TAU3, 1.0)
    t0, s0 = oracle_lib.emission_time(1, 0, 50_000, TAU1, TAU3, 0.0)
    assert s1.all() and not s0.any()
    # same uniforms, so the two samples differ exactly by the ratio of the constants
    assert np.allclose(t0 / t1, TAU3 / TAU1, rtol=1e-12)


def test_time_quantile_hand_computed():
    q = pytest.importorskip("oracle").time_quantile
    # 10 photons in bin 1 of width 1 ns: 9 of them are reached 0.9 of the way in
    assert q(np.array([[0, 10, 0, 0]]), 1.0, 0.9)[0] == pytest.approx(1.9)
    # 4 + 4 + 2 photons, q = 0.5: target 5 falls 1/4 into bin 1 (width 2 ns)
    assert q(np.array([[4, 4, 2, 0]]), 2.0, 0.5)[0] == pytest.approx(2.5)
    # q = 1 ends at the upper edge of the last occupied bin
    assert q(np.array([[1, 0, 3, 0, 0]]), 0.5, 1.0)[0] == pytest.approx(1.5)
    # empty events give NaN; a quantile in the open last bin gives inf
    r = q(np.array([[0, 0, 0], [1, 0, 9]]), 1.0, 0.9)
    assert math.isnan(r[0]) and math.isinf(r[1])


def test_t90_of_the_decay_profile(oracle_lib):
    """The t90 rule applied to a histogram of sampled emission times gives the
    analytic 90 % quantile of the two-component profile."""
    n, bin_ns = 400_000, 0.25
    t, _ = oracle_lib.emission_time(seed=11, pid0=0, n=n, tau_singlet=TAU1, tau_triplet=TAU3,
                                    singlet_fraction=FS)
    rec = np.zeros(n, dtype=oracle_lib.RECORD_DTYPE)
    rec["flag"] = oracle_lib.F_DETECT
    rec["time"] = t
    h = oracle_lib.time_histogram(rec, 1, 2000, bin_ns)
    assert h.sum() == n
    t90 = oracle_lib.time_quantile(h, bin_ns, 0.9)[0]
    exact = optimize.brentq(lambda x: mixture_cdf(x) - 0.9, 0.0, 500.0)
    pdf = FS / TAU1 * math.exp(-exact / TAU1) + (1 - FS) / TAU3 * math.exp(-exact / TAU3)
    sigma = math.sqrt(0.9 * 0.1 / n) / pdf
    assert abs(t90 - exact) < 5 * sigma + bin_ns / 4


def _slab_direct(oracle_lib, time_profile):
    mesh = W.slab()
    n = 4000
    pos = np.tile([0.0, 0.0, -0.05], (n, 1))
    dirs = np.tile([0.0, 0.0, 1.0], (n, 1))
    pols = np.tile([1.0, 0.0, 0.0], (n, 1))
    src = W.explicit_sources(pos, dirs, pols, medium=0)
    if time_profile:
        src = W.with_scintillation(src)
    rec = oracle_lib.run(oracle_lib.Scene(mesh), src, seed=5)["records"]
    # straight through: interface, quartz front, detected behind the quartz
    direct = ((rec["flag"] & 0xFF) == oracle_lib.F_DETECT) & (rec["sensor"] == 0) & (rec["steps"] == 3)
    return rec, direct


def test_time_of_flight_closed_form(oracle_lib):
    rec, direct = _slab_direct(oracle_lib, False)
    assert direct.sum() > 3000
    flight = (0.05 * 1.69 + W.SLAB_GAP * 1.00 + W.SLAB_QUARTZ_T * 1.60) / C_M_PER_NS
    # the 2 um restart offsets at the three crossings shorten the path by < 1e-5 m
    assert np.allclose(rec["time"][direct], flight, rtol=1e-4)


def test_emission_time_adds_to_flight(oracle_lib):
    rec0, d0 = _slab_direct(oracle_lib, False)
    rec1, d1 = _slab_direct(oracle_lib, True)
    # the emission-time draw has a Philox block of its own: histories are unchanged
    assert np.array_equal(d0, d1)
    assert np.array_equal(rec0["flag"], rec1["flag"]) and np.array_equal(rec0["pos"], rec1["pos"])
    t_emit, _ = oracle_lib.emission_time(5, 0, len(rec1), TAU1, TAU3, FS)
    assert np.allclose(rec1["time"] - t_emit, rec0["time"], rtol=0, atol=1e-9)


def test_loss_table_bulk_absorption_closed_form(oracle_lib):
    """Photons from the centre of an absorbing 1 m cube toward a face 0.5 m away
    are absorbed in the bulk with probability 1 - exp(-0.5 / L_abs)."""
    lab = 0.3
    mesh = W.disk_box()
    mesh = dataclasses.replace(mesh, materials=[W.Material(1.69, lab, W.INF)])
    n = 40_000
    src = W.explicit_sources(np.zeros((n, 3)), np.tile([1.0, 0, 0], (n, 1)),
                             np.tile([0, 0, 1.0], (n, 1)))
    rec = oracle_lib.run(oracle_lib.Scene(mesh), src, seed=9)["records"]
    groups = mesh.solid
    tab = oracle_lib.loss_table(rec, groups, int(groups.max()) + 1, len(mesh.materials))
    assert tab.sum() == n
    box = mesh.solid_names.index("box")
    n_groups = int(groups.max()) + 1
    bulk = tab[n_groups + 0, oracle_lib.F_BULK_ABSORB]
    p = 1.0 - math.exp(-0.5 / lab)
    assert abs(bulk / n - p) < 5 * binom_sigma(p, n)
    assert tab[box, oracle_lib.F_SURFACE_ABSORB] == n - bulk


def test_loss_table_partitions_the_photons(oracle_lib):
    wl = W.small_tpc(photons_per_point=2_000)
    mesh = wl.mesh
    rec = oracle_lib.run(oracle_lib.Scene(mesh), wl.sources, seed=2)["records"]
    ng = int(mesh.solid.max()) + 1
    tab = oracle_lib.loss_table(rec, mesh.solid, ng, len(mesh.materials))
    fl = rec["flag"] & 0xFF
    assert tab.sum() == len(rec)
    assert np.array_equal(tab.sum(axis=0), np.bincount(fl, minlength=8))
    # photons ending on a surface are booked under the solid of their last triangle
    surf = (fl >= 1) & (fl <= 3)
    assert np.array_equal(tab[:ng].sum(axis=1), np.bincount(mesh.solid[rec["last_tri"][surf]],
                                                            minlength=ng))
    assert tab[ng:, 1:4].sum() == 0 and tab[:ng, 4:].sum() == 0
