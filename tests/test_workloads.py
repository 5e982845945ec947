"""Invariants of the synthetic input generators (no GPU; the variant
consistency check runs photons through the oracle)."""
import math

import numpy as np
import pytest

from paper_2203_14354_amd import workloads as W
from tests.helpers import closed_edges_ok


def _sel(m, *names):
    return np.isin(m.solid, [m.solid_names.index(n) for n in names])


def test_tpc1_counts_and_closed_wall():
    m = W.tpc1()
    assert m.n_triangles == 4128 and m.n_sensors == 38
    assert closed_edges_ok(m.triangles[_sel(m, "wall", "cap_top", "cap_bottom")])
    # sensors: 48-gon fans of 36 mm diameter, 0.5 mm in front of the caps, facing inward
    n = m.normals()
    top = _sel(m, "sensors_top")
    bot = _sel(m, "sensors_bottom")
    assert np.allclose(n[top], [0, 0, -1]) and np.allclose(n[bot], [0, 0, 1])
    assert np.bincount(m.sensor[m.sensor >= 0]).tolist() == [48] * 38
    assert np.allclose(np.abs(m.vertices[m.triangles[top | bot]][:, :, 2]), 0.0995)
    # wall and caps point outward
    c = m.vertices[m.triangles].mean(axis=1)
    w = _sel(m, "wall")
    assert np.all(np.einsum("ij,ij->i", n[w], c[w] * [1, 1, 0]) > 0)
    # the outer ring of sensors stays inside the cylinder
    r = np.hypot(m.vertices[m.triangles[top]][..., 0], m.vertices[m.triangles[top]][..., 1])
    assert r.max() < W.TPC1_R
    mp = W.tpc1(plane=True)
    assert mp.n_triangles == 4256
    assert mp.surfaces[2].grad_param == W.GRAD_TRANSPARENCY


def test_darwin_counts_and_solids():
    m = W.darwin()
    assert 4.5e5 < m.n_triangles < 5.0e5
    assert m.n_sensors == 1778  # 889 per array at 80 mm hexagonal pitch
    assert closed_edges_ok(m.triangles[_sel(m, "wall_liquid", "wall_gas", "cap_top",
                                              "cap_bottom")])
    # every quartz window (front + side + photocathode + annulus) is a closed solid
    per = 192
    win = _sel(m, "window_bottom", "pmt_cap_bottom", "photocathode_bottom")
    tri = m.triangles[win]
    assert len(tri) == 889 * per
    for k in (0, 444, 888):
        assert closed_edges_ok(tri[k * per:(k + 1) * per], oriented=False)
    # media: quartz is on the inner side of the front face and the outer side of the cathode
    pc = _sel(m, "photocathode_top", "photocathode_bottom")
    assert np.all(m.mat_outer[pc] == 2) and np.all(m.surface[pc] == 3)
    wf = _sel(m, "window_top")
    assert np.all(m.mat_inner[wf] == 2) and np.all(m.mat_outer[wf] == 1)
    wb = _sel(m, "window_bottom")
    assert np.all(m.mat_outer[wb] == 0)
    # the liquid surface shares the wall ring at +2 mm (no gap between the media)
    iface = m.triangles[_sel(m, "interface")]
    wall = m.triangles[_sel(m, "wall_liquid", "wall_gas")]
    centre = np.argmax(np.bincount(iface.ravel()))
    ring = np.setdiff1d(np.unique(iface), [centre])
    assert len(ring) == 256
    assert np.all(np.isin(ring, wall))
    assert np.allclose(m.vertices[np.unique(iface)][:, 2], np.float32(W.DARWIN_Z_IFACE))
    # electrodes at the table's heights; strip segments no longer than 4 cm
    for name, z in (("electrode_gate", 0.0), ("electrode_cathode", -2.598),
                    ("electrode_bottom_screen", -2.678)):
        t = m.triangles[_sel(m, name)]
        v = m.vertices[t]
        assert np.allclose(v[..., 2], np.float32(z))
        assert (v[..., 0].max(axis=1) - v[..., 0].min(axis=1)).max() <= 0.04 + 1e-6
    # transparency of the strip planes ~ 0.9 (strip width = 10 % of the pitch)
    g = m.vertices[m.triangles[_sel(m, "electrode_gate")]].astype(np.float64)
    area = 0.5 * np.linalg.norm(np.cross(g[:, 1] - g[:, 0], g[:, 2] - g[:, 0]), axis=1).sum()
    assert abs(area / (math.pi * W.DARWIN_STRIP_RMAX ** 2) - 0.1) < 0.005
    # photocathodes at -2.693 m (bottom) as in the table of z coordinates
    assert np.allclose(m.vertices[m.triangles[_sel(m, "photocathode_bottom")]][..., 2],
                       np.float32(-2.693))


def test_darwin_sources_inside_active_volume():
    wl = W.darwin_tpc(n_photons=10)
    s = wl.sources
    # the inscribed 256-gon's edges lie at r cos(pi/256) > source radius
    assert W.DARWIN_R_WALL * math.cos(math.pi / 256) > s.cyl_radius
    assert W.DARWIN_Z_CATHODE < s.cyl_zlo < s.cyl_zhi < W.DARWIN_Z_GATE


def test_batched_s1_counts():
    wl = W.batched_s1()
    c = np.diff(wl.sources.offsets)
    assert len(c) == 4096 and c.min() >= 100 and c.max() <= 100_000
    assert 2500 <= np.median(c) <= 3500
    assert 1.5e7 < wl.sources.n_photons < 3.5e7
    assert wl.sources.n_events == 4096


def test_lce_map_cells():
    pos = W.equal_volume_cell_centroids(4, 4, 4, 0.099, -0.098, 0.098)
    assert pos.shape == (64, 3)
    r = np.hypot(pos[:, 0], pos[:, 1])
    assert r.max() < 0.099 and np.abs(pos[:, 2]).max() < 0.098
    # equal volumes: radial edges uniform in r^2
    big = W.equal_volume_cell_centroids(64, 64, 64, 0.099, -0.098, 0.098)
    assert big.shape == (64 ** 3, 3)


def test_inputs_are_seeded():
    a = W.small_tpc().sources.positions
    b = W.small_tpc().sources.positions
    assert np.array_equal(a, b)
    c = W.small_tpc(seed=1).sources.positions
    assert not np.array_equal(a, c)


def test_darwin_design_variants():
    """The paper's design variants (section "Alternative designs") on the same
    generator: what changes and what does not."""
    base = W.darwin()
    # reflective coatings: only the electrode surfaces change
    for coat, solids in (("gate", ["electrode_gate"]),
                         ("all", ["electrode_gate", "electrode_cathode", "electrode_bottom_screen"])):
        m = W.darwin(coating=coat)
        assert np.array_equal(m.triangles, base.triangles)
        changed = m.surface != base.surface
        assert np.array_equal(changed, _sel(m, *solids))
        s = m.surfaces[m.surface[changed][0]]
        assert s.r_specular + s.r_diffuse == pytest.approx(0.90)
        assert s.r_specular == pytest.approx(0.85)
    # single phase: no gas anywhere, no interface, the gas wall becomes liquid PTFE
    m = W.darwin(single_phase=True)
    assert not np.any(m.mat_inner == 1) and not np.any(m.mat_outer == 1)
    assert "interface" not in m.solid_names
    assert m.n_triangles == base.n_triangles - 256
    # no bottom array: the bottom PTFE (0.99) stays, 889 sensors remain
    m = W.darwin(bottom_array=False)
    assert m.n_sensors == 889 and "photocathode_bottom" not in m.solid_names
    assert np.bincount(W.darwin_array_channels(m)).tolist() == [889]
    # 4-pi: 6,480 square PMTs or 87,120 quad SiPMs on 24 plates behind 92 FSRs
    for kind, n_side, fsr in (("pmt2", 6480, "copper"), ("pmt2", 6480, None), ("sipm", 87120, "coated")):
        m = W.darwin(side_array=kind, fsr=fsr)
        assert np.bincount(W.darwin_array_channels(m)).tolist() == [889, 889, n_side]
        assert "wall_liquid" not in m.solid_names
        n_fsr = int(_sel(m, "fsr").sum()) if "fsr" in m.solid_names else 0
        assert n_fsr == (92 * 4 * 2 * 256 if fsr else 0)
        # the side sensors sit between the rings and the plates, facing the axis
        side = _sel(m, "side_photocathode" if kind == "pmt2" else "side_sipm")
        c = m.vertices[m.triangles[side]].mean(axis=1)
        r = np.hypot(c[:, 0], c[:, 1])
        assert r.min() > W.DARWIN_R_WALL + W.FSR_WIDTH and r.max() < W.SIDE_OUTER_R
        assert np.all(np.einsum("ij,ij->i", m.normals()[side], c * [1, 1, 0]) < 0)
        assert np.all((c[:, 2] > W.DARWIN_Z_BOTCAP) & (c[:, 2] < W.DARWIN_Z_IFACE))
    assert closed_edges_ok(W.darwin(side_array="pmt2").triangles[
        _sel(W.darwin(side_array="pmt2"), "fsr")])


@pytest.mark.parametrize("kw", [dict(coating="all"), dict(single_phase=True),
                                dict(bottom_array=False), dict(side_array="pmt2"),
                                dict(side_array="sipm", fsr=None)])
def test_darwin_variants_are_consistent_meshes(kw):
    """Photons through each variant (oracle, 3,000 photons): every one ends
    with a valid terminal flag, none escapes the closed detector and none
    meets a triangle whose media disagree with the tracked one."""
    import oracle
    m = W.darwin(**kw)
    sc = oracle.Scene(m, channel_of_sensor=W.darwin_array_channels(m), n_channels=3, use_bvh=True)
    rec = oracle.run(sc, W.darwin_tpc(n_photons=3000, mesh=m).sources, seed=3)["records"]
    fl = rec["flag"] & 0xFF
    assert np.all((fl >= 1) & (fl <= 4))
    assert not np.any(rec["flag"] & oracle.F_GEOMETRY_ERROR)
