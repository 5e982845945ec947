"""Pins of the oracle's outgoing polarization after a boundary event.

The paper computes reflection and refraction from the refractive indices at
the quartz / LXe / GXe boundaries and checks refraction and angle-dependent
reflection against an independent simulator (sections "Optical properties"
and "Comparison of Chroma and Geant4"); it fixes no polarization convention.
The oracle keeps each photon linearly polarized and splits it into s and p
parts (s along d x n, p along s x d for every wave) with real amplitude
coefficients.  These tests pin what it returns against physics computed here
without any Fresnel formula: the reflected and transmitted plane waves from
Maxwell's boundary conditions solved as a linear system
(``helpers.plane_wave_boundary``), energy flux conservation, Brewster's
angle, and Fresnel's sine/tangent laws in Hecht's form.  A photon's linear
polarization is an axis: the oracle's unit vector must be parallel or
antiparallel to the physical field.
"""
import math

import numpy as np
import pytest

from tests.helpers import plane_wave_boundary, poynting_z

N_LXE, N_GXE, N_QUARTZ = 1.69, 1.00, 1.60
Z = np.array([0.0, 0.0, 1.0])


def _incident(theta_deg, psi_deg, tilt=0.0):
    """Direction at incidence theta on the plane z = 0 (travelling down, the
    plane of incidence rotated by `tilt` about z), field at angle psi from the
    s axis (s = d x n normalized, p = s x d)."""
    t, a = math.radians(theta_deg), math.radians(tilt)
    d = np.array([math.sin(t) * math.cos(a), math.sin(t) * math.sin(a), -math.cos(t)])
    sv = np.cross(d, Z)
    s = sv / np.linalg.norm(sv) if np.linalg.norm(sv) > 1e-9 else np.array([math.sin(a), -math.cos(a), 0.0])
    p = np.cross(s, d)
    ps = math.radians(psi_deg)
    return d, math.cos(ps) * s + math.sin(ps) * p, s


def _parallel(u, v, tol):
    """|u x v| <= tol |u| |v| (an axis: either orientation)."""
    v = np.asarray(v)
    if np.iscomplexobj(v):
        # a linearly polarized wave: one global phase makes it real
        k = int(np.argmax(np.abs(v)))
        v = (v * np.exp(-1j * np.angle(v[k]))).real
    return np.linalg.norm(np.cross(u, v)) <= tol * np.linalg.norm(u) * np.linalg.norm(v)


def test_maxwell_solver_conserves_energy_and_reduces_to_normal_incidence():
    """The pinning tool itself: lossless interfaces conserve the normal energy
    flux, and at normal incidence the reflected field is (n1 - n2)/(n1 + n2)
    times the incident one."""
    rng = np.random.default_rng(0)
    for n1, n2 in ((N_LXE, N_GXE), (N_LXE, N_QUARTZ), (N_GXE, N_LXE), (N_GXE, N_QUARTZ)):
        tc = math.degrees(math.asin(min(1.0, n2 / n1)))
        for _ in range(20):
            th = rng.uniform(0, min(tc - 0.5, 85.0))
            d, e, _ = _incident(th, rng.uniform(0, 180), rng.uniform(0, 360))
            d_r, Er, kt, Et = plane_wave_boundary(d, e, Z, n1, n2)
            fi = poynting_z(n1 * d, e.astype(complex), Z)
            fr = poynting_z(n1 * d_r, Er, Z)
            ft = poynting_z(kt * n2, Et, Z)
            # fluxes along +z: incident and transmitted downward, reflected upward
            assert fi < 0 and ft < 0 and fr >= 0
            assert abs(fi + fr - ft) < 1e-12 * abs(fi)
            assert abs(np.linalg.norm(Er) ** 2 - fr / -fi) < 1e-12
        d, e, _ = _incident(0.0, 30.0)
        _, Er, _, _ = plane_wave_boundary(d, e, Z, n1, n2)
        assert np.allclose(Er, (n1 - n2) / (n1 + n2) * e, atol=1e-13)


CASES = ([(N_LXE, N_GXE, th) for th in (5.0, 15.0, 25.0, 30.6129, 34.0)]
         + [(N_LXE, N_QUARTZ, th) for th in (10.0, 30.0, 50.0, 65.0, 70.0)]
         + [(N_GXE, N_LXE, th) for th in (20.0, 45.0, 60.0, 80.0)]
         + [(N_GXE, N_QUARTZ, th) for th in (12.0, 58.0)])


@pytest.mark.parametrize("n1,n2,theta", CASES)
def test_fresnel_outgoing_polarization_matches_maxwell(oracle_lib, n1, n2, theta):
    """Reflected and refracted photon: direction and polarization axis of the
    plane wave Maxwell's boundary conditions give, and the reflection
    probability equal to the reflected power |E_r|^2; for pure s, pure p and
    mixed inputs, in planes of incidence at several azimuths."""
    for psi in (0.0, 90.0, 30.0, 60.0, 135.0):
        for tilt in (0.0, 77.0):
            d, e, _ = _incident(theta, psi, tilt)
            d_r, Er, kt, Et = plane_wave_boundary(d, e, Z, n1, n2)
            R = float(np.linalg.norm(Er) ** 2)
            # u just below R reflects, just above transmits
            if R > 1e-12:
                tr, dd, ee = oracle_lib.boundary(0, d, e, Z, n1, n2, u=R * (1 - 1e-9))
                assert not tr, (psi, tilt)
                assert np.allclose(dd, d_r, atol=1e-12)
                assert _parallel(ee, Er, 1e-9), (psi, tilt, ee, Er)
            tr, dd, ee = oracle_lib.boundary(0, d, e, Z, n1, n2, u=min(R * (1 + 1e-9) + 1e-15, 0.999999))
            assert tr, (psi, tilt)
            assert np.allclose(dd, kt.real, atol=1e-12)
            assert _parallel(ee, Et, 1e-9), (psi, tilt, ee, Et)


@pytest.mark.parametrize("n1,n2", [(N_LXE, N_GXE), (N_LXE, N_QUARTZ), (N_GXE, N_LXE)])
def test_brewster_reflection_is_pure_s(oracle_lib, n1, n2):
    """At Brewster's angle tan(theta_B) = n2/n1 every reflected photon is
    s-polarized, whatever its incoming polarization."""
    tb = math.degrees(math.atan(n2 / n1))
    rng = np.random.default_rng(3)
    for _ in range(50):
        d, e, s = _incident(tb, rng.uniform(5, 175), rng.uniform(0, 360))
        tr, _, ee = oracle_lib.boundary(0, d, e, Z, n1, n2, u=1e-9)
        assert not tr
        assert _parallel(ee, s, 1e-9)


@pytest.mark.parametrize("n1,n2,theta", [(N_LXE, N_GXE, 20.0), (N_LXE, N_QUARTZ, 45.0),
                                         (N_GXE, N_LXE, 50.0)])
def test_pure_s_and_pure_p_stay_pure(oracle_lib, n1, n2, theta):
    """An s-polarized photon stays perpendicular to the plane of incidence and
    a p-polarized one stays in it, after reflection and after refraction."""
    for psi in (0.0, 90.0):
        d, e, s = _incident(theta, psi, 33.0)
        for u in (1e-9, 0.999999):
            _, dd, ee = oracle_lib.boundary(0, d, e, Z, n1, n2, u=u)
            if psi == 0.0:
                assert _parallel(ee, s, 1e-12)
            else:
                assert abs(np.dot(ee, s)) < 1e-12
                assert abs(np.dot(ee, dd)) < 1e-12


def _hecht(theta_i, n1, n2):
    """Fresnel's laws in the sine/tangent form (Hecht, Optics, ch. 4):
    r_s = -sin(ti - tt)/sin(ti + tt), r_p = tan(ti - tt)/tan(ti + tt),
    t_s = 2 sin(tt) cos(ti)/sin(ti + tt),
    t_p = 2 sin(tt) cos(ti)/(sin(ti + tt) cos(ti - tt))."""
    tt = math.asin(n1 * math.sin(theta_i) / n2)
    a, b = theta_i - tt, theta_i + tt
    return (-math.sin(a) / math.sin(b), math.tan(a) / math.tan(b),
            2 * math.sin(tt) * math.cos(theta_i) / math.sin(b),
            2 * math.sin(tt) * math.cos(theta_i) / (math.sin(b) * math.cos(a)))


@pytest.mark.parametrize("n1,n2,theta", [(N_LXE, N_GXE, t) for t in (8.0, 17.0, 24.0, 29.0, 35.0)]
                         + [(N_LXE, N_QUARTZ, t) for t in (10.0, 25.0, 40.0, 55.0, 68.0)])
def test_amplitude_ratios_follow_sine_tangent_laws(oracle_lib, n1, n2, theta):
    """For a mixed input a_s s + a_p p, the outgoing p:s component ratio is
    (r_p a_p):(r_s a_s) after reflection and (t_p a_p):(t_s a_s) after
    refraction, with Hecht's sine/tangent forms, in the basis s = d x n,
    p = s x d of each wave (n toward the incident side)."""
    rs, rp, ts, tp = _hecht(math.radians(theta), n1, n2)
    for psi in (25.0, 70.0, 120.0):
        d, e, s = _incident(theta, psi)
        a_s, a_p = math.cos(math.radians(psi)), math.sin(math.radians(psi))
        R = (a_s * rs) ** 2 + (a_p * rp) ** 2
        tr, dr, er = oracle_lib.boundary(0, d, e, Z, n1, n2, u=R * (1 - 1e-9))
        assert not tr
        pr = np.cross(s, dr)
        assert abs(np.dot(er, pr) * (rs * a_s) - np.dot(er, s) * (rp * a_p)) < 1e-12
        tr, dt, et = oracle_lib.boundary(0, d, e, Z, n1, n2, u=R * (1 + 1e-9) + 1e-15)
        assert tr
        pt = np.cross(s, dt)
        assert abs(np.dot(et, pt) * (ts * a_s) - np.dot(et, s) * (tp * a_p)) < 1e-12
        # and the reflection probability is the reflected power
        assert abs(R - (a_s ** 2 * rs ** 2 + a_p ** 2 * rp ** 2)) < 1e-15


@pytest.mark.parametrize("theta", [40.0, 55.0, 70.0, 85.0])
def test_total_internal_reflection_mirrors_polarization(oracle_lib, theta):
    """Above the critical angle (36.28 deg on LXe/GXe) every photon is
    reflected; the reading without a TIR phase reflects the polarization as
    a perfect mirror does: the tangential field is reversed and the normal
    field kept (up to the axis orientation, E_r = -(e_t) + e_n)."""
    rng = np.random.default_rng(int(theta))
    for _ in range(20):
        d, e, _ = _incident(theta, rng.uniform(0, 180), rng.uniform(0, 360))
        tr, dr, er = oracle_lib.boundary(0, d, e, Z, N_LXE, N_GXE, u=rng.uniform(0, 1))
        assert not tr
        assert np.allclose(dr, d - 2 * np.dot(d, Z) * Z, atol=1e-12)
        mirror_field = -(e - np.dot(e, Z) * Z) + np.dot(e, Z) * Z
        assert _parallel(er, mirror_field, 1e-12)


def _model_coefficients(model, d, s, n1, n_re, n_im, film_n, film_d_nm, lam):
    """r_s and r_p of a complex-index substrate (model 1) or of a film on it
    (model 2), from Maxwell's boundary conditions, in the basis s, p = s x d
    of each wave."""
    layers = [(film_n, film_d_nm)] if model == 2 else []
    p_in = np.cross(s, d)
    d_r, Er_s, _, _ = plane_wave_boundary(d, s, Z, n1, complex(n_re, n_im), layers, lam)
    _, Er_p, _, _ = plane_wave_boundary(d, p_in, Z, n1, complex(n_re, n_im), layers, lam)
    return d_r, np.dot(Er_s, s), np.dot(Er_p, np.cross(s, d_r))


MODEL_CASES = [
    (1, N_LXE, 0.81, 1.86, 0.0, 0.0),      # silicon from the liquid (section "Alternative designs")
    (1, N_GXE, 0.81, 1.86, 0.0, 0.0),
    (1, N_LXE, 0.11, 2.00, 0.0, 0.0),      # an aluminium-like metal
    (2, N_LXE, 0.11, 2.00, 1.42, 25.0),    # Al/MgF2-like coating
    (2, N_GXE, 0.11, 2.00, 1.42, 60.0),
    (2, N_LXE, 1.60, 0.00, 1.42, 40.0),    # a film on a dielectric
]


@pytest.mark.parametrize("model,n1,n_re,n_im,film_n,film_d", MODEL_CASES)
def test_complex_and_film_reflection_match_maxwell(oracle_lib, model, n1, n_re, n_im, film_n,
                                                   film_d):
    """Complex-index and thin-film surfaces at oblique incidence: the power
    reflectances |r_s|^2, |r_p|^2 equal those of Maxwell's boundary conditions
    (the film as a layer with its own up- and down-going waves, no Airy
    formula), the reflection probability is a_s^2 |r_s|^2 + a_p^2 |r_p|^2, and
    the reflected polarization is the reading's |r_s| sgn(Re r_s) a_s s +
    |r_p| sgn(Re r_p) a_p p."""
    lam = 174.8
    for theta in (0.0, 20.0, 45.0, 60.0, 75.0, 85.0):
        cos_i = math.cos(math.radians(theta))
        Rs_o, Rp_o = oracle_lib.surface_reflectance(model, n1, n_re, n_im, film_n, film_d, lam,
                                                    cos_i=[cos_i])
        for psi in (0.0, 90.0, 35.0, 110.0):
            d, e, s = _incident(theta, psi, 21.0)
            d_r, rs, rp = _model_coefficients(model, d, s, n1, n_re, n_im, film_n, film_d, lam)
            assert abs(Rs_o[0] - abs(rs) ** 2) < 1e-12 and abs(Rp_o[0] - abs(rp) ** 2) < 1e-12
            if theta == 0.0:
                continue  # s is taken along the polarization at normal incidence
            a_s, a_p = math.cos(math.radians(psi)), math.sin(math.radians(psi))
            R = a_s ** 2 * abs(rs) ** 2 + a_p ** 2 * abs(rp) ** 2
            refl, dr, er = oracle_lib.model_boundary(model, d, e, Z, n1, n_re, n_im, film_n,
                                                     film_d, lam, u=R * (1 - 1e-9))
            assert refl
            assert np.allclose(dr, d_r, atol=1e-12)
            want = (abs(rs) * math.copysign(1, rs.real) * a_s * s
                    + abs(rp) * math.copysign(1, rp.real) * a_p * np.cross(s, d_r))
            assert _parallel(er, want, 1e-9), (theta, psi, er, want)
            refl, _, _ = oracle_lib.model_boundary(model, d, e, Z, n1, n_re, n_im, film_n, film_d,
                                                   lam, u=R * (1 + 1e-9) + 1e-15)
            assert not refl


def test_fp32_build_follows_the_same_polarization(oracle_lib):
    """The FP32 diagnostic build computes the same boundary events to single
    precision."""
    for n1, n2, theta in ((N_LXE, N_GXE, 25.0), (N_LXE, N_QUARTZ, 50.0)):
        d, e, _ = _incident(theta, 40.0, 10.0)
        for u in (1e-6, 0.999):
            tr64, d64, e64 = oracle_lib.boundary(0, d, e, Z, n1, n2, u=u)
            tr32, d32, e32 = oracle_lib.boundary(0, d, e, Z, n1, n2, u=u, fp32=True)
            assert tr64 == tr32
            assert np.allclose(d64, d32, atol=2e-6) and np.allclose(e64, e32, atol=2e-6)
