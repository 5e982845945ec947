"""GPU parity of the wavelength-dependent optics (through the C ABI).

Bars: emission wavelengths within 2e-6 relative of the oracle's (FP32 vs FP64
of the same Box-Muller formula); complex-index and thin-film reflectances
within 2e-5 absolute (FP32 complex arithmetic; the film phase carries the
FP32 rounding of 2 pi d q / lambda); per photon, the same terminal flag, final
triangle, sensor and step count as the oracle for >= 99.9 % of photons on a
TPC with a dispersive medium, the Gaussian spectrum, silicon-like detecting
surfaces and a coated plane; the hit map identical to the histogram of the
GPU's own records.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2203_14354_amd import workloads as W
from tests.gpu_common import agreement, hist_of_detected, to_records

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_14354_amd import runtime
    return runtime


def test_wavelength_sampler_matches_oracle(rt):
    n = 200_000
    g = rt.sample_wavelength(6, 500, n, W.SCINT_WAVELENGTH_NM, W.SCINT_FWHM_NM).cpu().numpy()
    o = oracle.wavelength(6, 500, n, W.SCINT_WAVELENGTH_NM, W.SCINT_FWHM_NM)
    assert np.allclose(g, o, rtol=2e-6, atol=0)


@pytest.mark.parametrize("params", [
    dict(model=1, n1=1.69, n_re=W.SILICON_N, n_im=W.SILICON_K),
    dict(model=1, n1=1.69, n_re=1.0, n_im=0.0),           # dielectric, with total reflection
    dict(model=1, n1=1.0, n_re=0.11, n_im=2.0),
    dict(model=2, n1=1.69, n_re=0.11, n_im=2.0, film_n=1.42, film_d_nm=25.0),
    dict(model=2, n1=1.69, n_re=W.SILICON_N, n_im=W.SILICON_K, film_n=1.2, film_d_nm=300.0),
    dict(model=2, n1=1.0, n_re=1.9, n_im=0.0, film_n=1.38, film_d_nm=174.8 / (4 * 1.38)),
])
def test_reflectance_matches_oracle(rt, params):
    c = np.concatenate([np.linspace(1e-4, 1.0, 4001), [1.0]]).astype(np.float32)
    p = dict(params)
    model = p.pop("model")
    rs, rp = rt.surface_reflectance(model, p["n1"], p["n_re"], p["n_im"],
                                    torch.from_numpy(c).cuda(), film_n=p.get("film_n", 0.0),
                                    film_d_nm=p.get("film_d_nm", 0.0), lam=174.8)
    ors, orp = oracle.surface_reflectance(model, p["n1"], p["n_re"], p["n_im"],
                                          film_n=p.get("film_n", 0.0),
                                          film_d_nm=p.get("film_d_nm", 0.0), lam=174.8,
                                          cos_i=c.astype(np.float64))
    assert np.allclose(rs.cpu().numpy(), ors, atol=2e-5, rtol=0)
    assert np.allclose(rp.cpu().numpy(), orp, atol=2e-5, rtol=0)


def optics_tpc():
    """The small TPC with a dispersive LXe (index and Rayleigh length varying
    across the spectrum), silicon-like detecting sensors, and the transparent
    plane replaced by an Al/MgF2-like coated reflector."""
    mesh = W.tpc1(plane=True)
    table = np.array([[160.0, 1.75, 50.0, 0.30], [175.0, 1.69, 50.0, 0.40],
                      [190.0, 1.64, 60.0, 0.55]])
    mats = [dataclasses.replace(mesh.materials[0], dispersion=table)]
    surfs = list(mesh.surfaces)
    for i, s in enumerate(surfs):
        if s.p_detect > 0:  # the sensors
            surfs[i] = W.complex_surface(W.SILICON_N, W.SILICON_K, flags=s.flags)
        elif s.p_transmit > 0:  # the plane
            surfs[i] = W.thin_film_surface(1.42, 25.0, 0.11, 2.0)
    return dataclasses.replace(mesh, materials=mats, surfaces=surfs)


def test_transport_with_optics_matches_oracle(rt):
    mesh = optics_tpc()
    det = rt.Detector(mesh, device=0)
    src = W.with_spectrum(W.small_tpc(photons_per_point=10_000).sources)
    out = det.propagate(src, seed=17, records=True, grad_material=-1)
    torch.cuda.synchronize()
    g = to_records(out["records"])
    o = oracle.run(oracle.Scene(mesh), src, seed=17, grad_material=-1)["records"]
    assert np.allclose(g["wavelength"], o["wavelength"], rtol=2e-6)
    assert g["wavelength"].std() > 3.0  # the spectrum is on
    ag = agreement(g, o)
    assert ag.mean() >= 0.999, ag.mean()
    hm = out["hit_map"].cpu().numpy()
    assert np.array_equal(hm, hist_of_detected(g, 1, det.n_channels))
    assert hm.sum() > 0


def test_optics_validation(rt):
    from paper_2203_14354_amd._lib import XpError
    mesh = optics_tpc()
    det = rt.Detector(mesh, device=0)
    src = W.small_tpc(photons_per_point=10).sources
    # the gradient material (LXe) has a dispersion table
    with pytest.raises(XpError):
        det.propagate(src, seed=0, grad=True, grad_material=0)
    # a thin-film surface needs a wavelength
    with pytest.raises(XpError):
        det.propagate(dataclasses.replace(src, wavelength_nm=0.0), seed=0, grad_material=-1)
