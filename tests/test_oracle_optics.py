"""Pins of the oracle's wavelength-dependent optics.

The Gaussian emission spectrum (section "Optical properties": mean 174.8 nm,
FWHM 10.2 nm), the interpolation of dispersion tables, and the reflectance of
surfaces given by a complex refractive index (the silicon of the 4-pi design:
n = 0.81, k = 1.86) or by a thin dielectric film on such a substrate (the
Al/MgF2 coatings of section "Alternative designs") are checked against the
paper's printed numbers, textbook closed forms (normal-incidence metal
reflectance, Brewster's angle, quarter- and half-wave layers) and limits.
None of these tests needs a GPU.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2203_14354_amd import workloads as W
from tests.helpers import binom_sigma

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_emission_spectrum(oracle_lib):
    lam = oracle_lib.wavelength(seed=4, pid0=0, n=200_000, mean=W.SCINT_WAVELENGTH_NM,
                                fwhm=W.SCINT_FWHM_NM)
    sigma = W.SCINT_FWHM_NM / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    assert stats.kstest(lam, "norm", args=(W.SCINT_WAVELENGTH_NM, sigma)).pvalue > 1e-3
    # the width is the FWHM: 76.1 % of a Gaussian lies within +- FWHM / 2
    inside = np.mean(np.abs(lam - W.SCINT_WAVELENGTH_NM) < W.SCINT_FWHM_NM / 2)
    assert abs(inside - 0.7610) < 5 * binom_sigma(0.761, len(lam))
    mono = oracle_lib.wavelength(seed=4, pid0=0, n=100, mean=174.8, fwhm=0.0)
    assert np.all(mono == np.float32(174.8))


def _dispersive_box(table):
    mesh = W.disk_box()
    mat = W.Material(1.69, W.INF, W.INF, dispersion=np.asarray(table, dtype=np.float64))
    return dataclasses.replace(mesh, materials=[mat])


def test_material_interpolation_hand_values(oracle_lib):
    inf = W.INF
    table = [[160.0, 1.80, 20.0, 0.2], [180.0, 1.60, inf, 0.4], [200.0, 1.50, 50.0, inf]]
    sc = oracle_lib.Scene(_dispersive_box(table))
    out = sc.material_at(0, [150.0, 160.0, 170.0, 175.0, 190.0, 210.0])
    # clamped below / at the first sample
    assert np.allclose(out[0], [1.80, 20.0, 0.2]) and np.allclose(out[1], [1.80, 20.0, 0.2])
    # midway 160..180: n = 1.70; 1/L_abs = (1/20 + 0) / 2 -> 40; 1/L_R = (5 + 2.5) / 2 -> 4/15
    assert np.allclose(out[2], [1.70, 40.0, 1.0 / 3.75])
    # 3/4 of the way: 1/L_abs = 0.05 / 4 -> 80
    assert np.allclose(out[3], [1.65, 80.0, 1.0 / (5.0 * 0.25 + 2.5 * 0.75)])
    # 180..200 midway: 1/L_abs = 0.01 -> 100; 1/L_R = 1.25 -> 0.8
    assert np.allclose(out[4], [1.55, 100.0, 0.8])
    assert out[5][0] == pytest.approx(1.50) and out[5][1] == pytest.approx(50.0)
    assert np.isinf(out[5][2])


def test_dispersive_bulk_absorption_closed_form(oracle_lib):
    """Photons at 170 nm toward a wall 0.5 m away through a medium whose
    absorption length is 0.2 m at 160 nm and infinite at 180 nm: L(170) = 0.4 m
    from the attenuation coefficient interpolated midway."""
    inf = W.INF
    mesh = _dispersive_box([[160.0, 1.69, 0.2, inf], [180.0, 1.69, inf, inf]])
    n = 40_000
    src = W.explicit_sources(np.zeros((n, 3)), np.tile([1.0, 0, 0], (n, 1)),
                             np.tile([0, 0, 1.0], (n, 1)))
    src = dataclasses.replace(src, wavelength_nm=170.0)
    rec = oracle_lib.run(oracle_lib.Scene(mesh), src, seed=3)["records"]
    assert np.all(rec["wavelength"] == np.float32(170.0))
    p = 1.0 - math.exp(-0.5 / 0.4)
    frac = np.mean((rec["flag"] & 0xFF) == oracle_lib.F_BULK_ABSORB)
    assert abs(frac - p) < 5 * binom_sigma(p, n)


def test_complex_index_reduces_to_dielectric_fresnel(oracle_lib):
    """k = 0: the paper's first validation check reflects 6.5 % at the LXe/GXe
    surface at normal incidence (printed), and s/p follow the dielectric laws."""
    g = json.load(open(os.path.join(GOLDEN, "paper_fresnel_worked_example.json")))
    rs, rp = oracle_lib.surface_reflectance(1, g["n_lxe"], g["n_gxe"], 0.0, cos_i=1.0)
    assert rs[0] == pytest.approx(rp[0])
    assert abs(rs[0] - g["reflected_at_lxe_gxe"]) <= g["printed_resolution"]
    # Brewster's angle, tan = n2 / n1: no p reflection
    n1, n2 = 1.0, 1.6
    cb = math.cos(math.atan(n2 / n1))
    rs, rp = oracle_lib.surface_reflectance(1, n1, n2, 0.0, cos_i=cb)
    assert rp[0] < 1e-20 and rs[0] > 0.1
    # beyond the critical angle (LXe -> GXe) every photon is reflected
    rs, rp = oracle_lib.surface_reflectance(1, 1.69, 1.0, 0.0, cos_i=math.cos(math.radians(75)))
    assert rs[0] == pytest.approx(1.0) and rp[0] == pytest.approx(1.0)


def test_metal_reflectance_closed_forms(oracle_lib):
    n1, n, k = 1.69, W.SILICON_N, W.SILICON_K
    rs, rp = oracle_lib.surface_reflectance(1, n1, n, k, cos_i=1.0)
    closed = ((n1 - n) ** 2 + k ** 2) / ((n1 + n) ** 2 + k ** 2)
    assert rs[0] == pytest.approx(closed, rel=1e-12) and rp[0] == pytest.approx(closed, rel=1e-12)
    # grazing incidence reflects everything; R stays within [0, 1]
    c = np.linspace(1e-9, 1.0, 2001)
    rs, rp = oracle_lib.surface_reflectance(1, n1, n, k, cos_i=c)
    assert rs[0] > 0.999999 and rp[0] > 0.999999
    assert np.all((rs >= 0) & (rs <= 1)) and np.all((rp >= 0) & (rp <= 1))
    # p falls below s at oblique incidence (pseudo-Brewster minimum)
    assert np.all(rp[1:-1] <= rs[1:-1] + 1e-12)


def test_thin_film_closed_forms(oracle_lib):
    lam = 174.8
    n1, nf, n2 = 1.0, 1.38, 1.90
    # zero thickness: the bare substrate, for a metal too
    for k in (0.0, 1.86):
        c = np.linspace(0.05, 1.0, 50)
        a = oracle_lib.surface_reflectance(2, 1.69, 0.81, k, film_n=1.42, film_d_nm=0.0, lam=lam,
                                           cos_i=c)
        b = oracle_lib.surface_reflectance(1, 1.69, 0.81, k, cos_i=c)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-15)
    # quarter-wave layer at normal incidence: ((n1 n2 - nf^2) / (n1 n2 + nf^2))^2
    rs, rp = oracle_lib.surface_reflectance(2, n1, n2, 0.0, film_n=nf, film_d_nm=lam / (4 * nf),
                                            lam=lam, cos_i=1.0)
    assert rs[0] == pytest.approx(((n1 * n2 - nf ** 2) / (n1 * n2 + nf ** 2)) ** 2, rel=1e-10)
    # half-wave layer: absent at normal incidence
    rs, _ = oracle_lib.surface_reflectance(2, n1, n2, 0.0, film_n=nf, film_d_nm=lam / (2 * nf),
                                           lam=lam, cos_i=1.0)
    bare, _ = oracle_lib.surface_reflectance(1, n1, n2, 0.0, cos_i=1.0)
    assert rs[0] == pytest.approx(bare[0], rel=1e-10)
    # a lossless stack reflects at most everything; a thick film from a denser
    # medium (evanescent in the film) still stays within [0, 1]
    rng = np.random.default_rng(0)
    for _ in range(50):
        c = rng.uniform(1e-3, 1.0, 20)
        rs, rp = oracle_lib.surface_reflectance(2, 1.69, rng.uniform(0.1, 3), rng.uniform(0, 3),
                                                film_n=rng.uniform(1.0, 2.0),
                                                film_d_nm=rng.uniform(0, 500), lam=174.8, cos_i=c)
        assert np.all((rs >= -1e-12) & (rs <= 1 + 1e-12)) and np.all((rp >= -1e-12) & (rp <= 1 + 1e-12))


def test_complex_surface_in_transport(oracle_lib):
    """Photons at normal incidence on a silicon-like detecting disk: a fraction
    R = ((n1 - n)^2 + k^2) / ((n1 + n)^2 + k^2) is reflected back into the
    absorbing box, the rest enters the disk and is detected."""
    mesh = W.disk_box()
    surfs = list(mesh.surfaces)
    surfs[0] = W.complex_surface(W.SILICON_N, W.SILICON_K)
    mesh = dataclasses.replace(mesh, surfaces=surfs)
    n = 40_000
    src = W.explicit_sources(np.zeros((n, 3)), np.tile([0, 0, 1.0], (n, 1)),
                             np.tile([1.0, 0, 0], (n, 1)))
    rec = oracle_lib.run(oracle_lib.Scene(mesh), src, seed=8)["records"]
    fl = rec["flag"] & 0xFF
    n1, nn, k = 1.69, W.SILICON_N, W.SILICON_K
    R = ((n1 - nn) ** 2 + k ** 2) / ((n1 + nn) ** 2 + k ** 2)
    det = np.mean(fl == oracle_lib.F_DETECT)
    assert abs(det - (1 - R)) < 5 * binom_sigma(1 - R, n)
    # reflected photons come straight back down with their polarization kept
    back = fl == oracle_lib.F_SURFACE_ABSORB
    assert np.all(rec["steps"][back] == 2)
    assert np.allclose(rec["dir"][back], [0, 0, -1], atol=1e-12)
    assert np.allclose(np.abs(rec["pol"][back][:, 0]), 1.0, atol=1e-12)
