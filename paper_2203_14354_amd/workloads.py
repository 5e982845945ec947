"""Seeded synthetic inputs: detector meshes, optical tables and source lists.

This module only *builds inputs*.  It holds none of the transport arithmetic
(no sampling of photon paths, no physics): both the HIP path and the CPU
oracle receive the arrays it returns, and nothing here is shared code between
them beyond these input arrays.

The real DARWIN CAD geometry is not public (Code and data availability
statement), so every detector below is synthetic and shaped after the paper:

* optical constants follow the "Optical properties" section (table
  ``tab:optical``): LXe n = 1.69, L_abs = 50 m, L_Rayleigh ~ 0.36-0.40 m;
  GXe n = 1.0, L_abs = 500 m, L_Rayleigh = 200 m; quartz n = 1.60, k = 0;
  PTFE R_total 0.99 in LXe and 0.80 in GXe with R_spec/R_diff = 0.05; SS
  R_total 0.30 with R_spec/R_diff = 2.
* the DARWIN-scale TPC follows the geometry section and table ``tab:z``:
  drift length 2598 mm, gate at z = 0, cathode at -2598 mm, bottom screen at
  -2678 mm, LXe/GXe boundary at +2 mm, bottom photocathodes at -2693 mm, 3-inch
  sensors with a 64 mm photocathode behind a 5 mm quartz window, hexagonal
  packing, wire electrodes of 5 mm (top) / 7.5 mm (bottom) pitch.

Conventions (shared by every consumer of these arrays):

* units are metres; vertices are float32, triangles int32 (nt, 3);
* the geometric normal (v1 - v0) x (v2 - v0) points to the triangle's *outer*
  side; ``mat_inner`` / ``mat_outer`` name the media on each side;
* ``surface`` = -1 means "no explicit surface" (a dielectric boundary when the
  refractive indices differ, else a pass-through);
* ``sensor`` = -1 means "not a photosensor".
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# ----------------------------------------------------------------------------
# optical tables
# ----------------------------------------------------------------------------

SURF_DETECT_FRONT_ONLY = 1  # detection only for photons arriving from the outer side

# gradient parameter tags (the four parameters of the differentiable run)
GRAD_ABS_LENGTH = 0
GRAD_RAYLEIGH_LENGTH = 1
GRAD_REFLECTIVITY = 2
GRAD_TRANSPARENCY = 3

INF = float("inf")


@dataclasses.dataclass
class Material:
    n: float
    abs_length: float
    rayleigh_length: float
    # optional dispersion table: rows (wavelength nm, n, L_abs, L_Rayleigh),
    # wavelengths ascending, at most 8 rows
    dispersion: Optional[np.ndarray] = None


@dataclasses.dataclass
class Surface:
    p_detect: float = 0.0
    p_absorb: float = 0.0
    r_diffuse: float = 0.0
    r_specular: float = 0.0
    p_transmit: float = 0.0
    grad_param: int = -1
    flags: int = 0
    # reflectance model: 0 explicit partition (above), 1 complex index
    # n_re + i n_im behind the surface, 2 a film (film_n, film_thickness_nm) on
    # that substrate
    model: int = 0
    n_re: float = 0.0
    n_im: float = 0.0
    film_n: float = 0.0
    film_thickness_nm: float = 0.0


def split_reflectivity(r_total: float, spec_over_diff: float):
    """R_spec, R_diff from a total reflectivity and a R_spec/R_diff ratio."""
    r_spec = r_total * spec_over_diff / (1.0 + spec_over_diff)
    r_diff = r_total / (1.0 + spec_over_diff)
    return r_spec, r_diff


def reflector(r_total: float, spec_over_diff: float, grad_param: int = -1) -> Surface:
    r_spec, r_diff = split_reflectivity(r_total, spec_over_diff)
    return Surface(p_absorb=1.0 - r_spec - r_diff, r_diffuse=r_diff, r_specular=r_spec,
                   grad_param=grad_param)


# best-guess values of table tab:optical (175 nm)
LXE = Material(1.69, 50.0, 0.40)
GXE = Material(1.00, 500.0, 200.0)
QUARTZ = Material(1.60, INF, INF)


def materials_array(mats: Sequence[Material]) -> np.ndarray:
    return np.array([[m.n, m.abs_length, m.rayleigh_length] for m in mats], dtype=np.float32)


def surfaces_array(surfs: Sequence[Surface]):
    p = np.array([[s.p_detect, s.p_absorb, s.r_diffuse, s.r_specular, s.p_transmit]
                  for s in surfs], dtype=np.float32).reshape(-1, 5)
    tags = np.array([[s.grad_param, s.flags, s.model] for s in surfs],
                    dtype=np.int32).reshape(-1, 3)
    optics = np.array([[s.n_re, s.n_im, s.film_n, s.film_thickness_nm] for s in surfs],
                      dtype=np.float32).reshape(-1, 4)
    return p, tags, optics


SURF_MODEL_EXPLICIT, SURF_MODEL_COMPLEX, SURF_MODEL_THIN_FILM = 0, 1, 2
# silicon at 175 nm (section "Alternative designs", optical table of the 4-pi
# design): n = 0.81, k = 1.86
SILICON_N, SILICON_K = 0.81, 1.86


def complex_surface(n_re, n_im, flags=0) -> Surface:
    """A surface whose reflectance follows from the complex index behind it."""
    return Surface(model=SURF_MODEL_COMPLEX, n_re=float(n_re), n_im=float(n_im), flags=flags)


def thin_film_surface(film_n, film_thickness_nm, n_re, n_im, flags=0) -> Surface:
    """A dielectric film of index film_n and the given thickness on a
    substrate of complex index n_re + i n_im."""
    return Surface(model=SURF_MODEL_THIN_FILM, n_re=float(n_re), n_im=float(n_im),
                   film_n=float(film_n), film_thickness_nm=float(film_thickness_nm), flags=flags)


# ----------------------------------------------------------------------------
# mesh container and builder
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Mesh:
    vertices: np.ndarray      # float32 (nv, 3)
    triangles: np.ndarray     # int32 (nt, 3)
    mat_inner: np.ndarray     # int32 (nt,)
    mat_outer: np.ndarray     # int32 (nt,)
    surface: np.ndarray       # int32 (nt,)
    sensor: np.ndarray        # int32 (nt,)
    materials: List[Material]
    surfaces: List[Surface]
    n_sensors: int
    name: str = ""
    solid: Optional[np.ndarray] = None   # int32 (nt,) component id (for bookkeeping only)
    solid_names: Optional[List[str]] = None

    @property
    def n_triangles(self) -> int:
        return int(self.triangles.shape[0])

    def normals(self) -> np.ndarray:
        v = self.vertices.astype(np.float64)
        t = self.triangles
        n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
        return n / np.linalg.norm(n, axis=1, keepdims=True)


class MeshBuilder:
    """Accumulates vertices and oriented triangles with per-triangle tags."""

    def __init__(self):
        self._v: List[np.ndarray] = []
        self._nv = 0
        self._t: List[np.ndarray] = []
        self._tags: List[np.ndarray] = []
        self.solid_names: List[str] = []

    def add_vertices(self, pts) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        idx = np.arange(self._nv, self._nv + len(pts), dtype=np.int64)
        self._v.append(pts)
        self._nv += len(pts)
        return idx

    def _vertex_array(self) -> np.ndarray:
        return np.concatenate(self._v, axis=0) if self._v else np.zeros((0, 3))

    def add_triangles(self, tris, outward, mat_inner, mat_outer, surface=-1, sensor=-1,
                      solid: str = ""):
        """Add triangles, flipping each so that its normal has a positive
        component along ``outward`` (one (3,) vector or one per triangle)."""
        tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3).copy()
        if len(tris) == 0:
            return
        v = self._vertex_array()
        n = np.cross(v[tris[:, 1]] - v[tris[:, 0]], v[tris[:, 2]] - v[tris[:, 0]])
        outward = np.broadcast_to(np.asarray(outward, dtype=np.float64), n.shape)
        flip = np.einsum("ij,ij->i", n, outward) < 0
        tris[flip, 1], tris[flip, 2] = tris[flip, 2].copy(), tris[flip, 1].copy()
        if solid not in self.solid_names:
            self.solid_names.append(solid)
        sid = self.solid_names.index(solid)
        cnt = len(tris)
        tags = np.stack([np.broadcast_to(np.asarray(x, dtype=np.int64), (cnt,))
                         for x in (mat_inner, mat_outer, surface, sensor, sid)], axis=1)
        self._t.append(tris)
        self._tags.append(tags)

    def build(self, materials, surfaces, n_sensors, name="") -> Mesh:
        v = self._vertex_array().astype(np.float32)
        t = np.concatenate(self._t).astype(np.int32)
        tags = np.concatenate(self._tags).astype(np.int32)
        return Mesh(vertices=v, triangles=t, mat_inner=tags[:, 0].copy(),
                    mat_outer=tags[:, 1].copy(), surface=tags[:, 2].copy(),
                    sensor=tags[:, 3].copy(), materials=list(materials),
                    surfaces=list(surfaces), n_sensors=int(n_sensors), name=name,
                    solid=tags[:, 4].copy(), solid_names=list(self.solid_names))


def _ring(nseg, radius, z, cx=0.0, cy=0.0, phase=0.0):
    a = phase + 2.0 * np.pi * np.arange(nseg) / nseg
    return np.stack([cx + radius * np.cos(a), cy + radius * np.sin(a), np.full(nseg, z)], axis=1)


def _fan(center_idx, ring_idx):
    n = len(ring_idx)
    return np.stack([np.full(n, center_idx), ring_idx, np.roll(ring_idx, -1)], axis=1)


def _band(ring_a, ring_b):
    """Quads between two rings of equal length, as two triangles each."""
    a0, a1 = ring_a, np.roll(ring_a, -1)
    b0, b1 = ring_b, np.roll(ring_b, -1)
    return np.concatenate([np.stack([a0, a1, b1], 1), np.stack([a0, b1, b0], 1)], 0)


def _annulus(inner_idx, outer_idx):
    return _band(inner_idx, outer_idx)


def hex_centres(pitch, r_max, rotate_30=False):
    """Hexagonally packed centres within radius r_max (centre at the origin)."""
    nmax = int(math.ceil(r_max / pitch)) + 2
    pts = []
    for j in range(-2 * nmax, 2 * nmax + 1):
        y = j * pitch * math.sqrt(3.0) / 2.0
        off = 0.5 * pitch if (j % 2) else 0.0
        for i in range(-nmax - 1, nmax + 2):
            x = i * pitch + off
            if x * x + y * y <= r_max * r_max + 1e-12:
                pts.append((x, y))
    pts = np.array(pts, dtype=np.float64)
    if rotate_30:
        pts = pts[:, ::-1].copy()
    order = np.lexsort((pts[:, 0], pts[:, 1]))
    return pts[order]


# ----------------------------------------------------------------------------
# small TPC (G-tpc1) -- used by the small-TPC, batched, differentiable and
# LCE-map workloads
# ----------------------------------------------------------------------------

TPC1_R = 0.10
TPC1_ZHALF = 0.10
TPC1_SENSOR_Z = 0.0995
TPC1_SENSOR_R = 0.018
TPC1_PITCH = 0.038
TPC1_PLANE_Z = 0.09


def tpc1_sensor_centres():
    """19 hexagonal positions: centre, 6 at one pitch, 12 in the second ring."""
    p = TPC1_PITCH
    pts = [(0.0, 0.0)]
    for k in range(6):
        a = math.radians(60 * k)
        pts.append((p * math.cos(a), p * math.sin(a)))
    for k in range(6):
        a = math.radians(60 * k)
        pts.append((2 * p * math.cos(a), 2 * p * math.sin(a)))
    for k in range(6):
        a = math.radians(60 * k + 30)
        r = p * math.sqrt(3.0)
        pts.append((r * math.cos(a), r * math.sin(a)))
    return np.array(pts)


def tpc1(plane: bool = False, qe: float = 0.3, ptfe_r: float = 0.95,
         plane_t: float = 0.9, lxe: Material = LXE) -> Mesh:
    """Closed PTFE cylinder r = 0.10 m, |z| <= 0.10 m, filled with LXe, with
    19 + 19 disk sensors 0.5 mm in front of the end caps.  4,128 triangles
    (4,256 with the transparent plane at z = +0.09 m)."""
    mb = MeshBuilder()
    LX = 0
    nseg, nband = 128, 8
    zs = np.linspace(-TPC1_ZHALF, TPC1_ZHALF, nband + 1)
    rings = [mb.add_vertices(_ring(nseg, TPC1_R, z)) for z in zs]
    v = mb._vertex_array()
    for b in range(nband):
        tri = _band(rings[b], rings[b + 1])
        c = v[tri].mean(axis=1)
        mb.add_triangles(tri, c * np.array([1, 1, 0]), LX, LX, surface=0, solid="wall")
    for z, ring, sgn in ((-TPC1_ZHALF, rings[0], -1.0), (TPC1_ZHALF, rings[-1], 1.0)):
        ci = mb.add_vertices([[0.0, 0.0, z]])[0]
        mb.add_triangles(_fan(ci, ring), [0, 0, sgn], LX, LX, surface=0,
                         solid="cap_top" if sgn > 0 else "cap_bottom")
    centres = tpc1_sensor_centres()
    sid = 0
    for z, inward in ((TPC1_SENSOR_Z, -1.0), (-TPC1_SENSOR_Z, 1.0)):
        for (cx, cy) in centres:
            ci = mb.add_vertices([[cx, cy, z]])[0]
            ring = mb.add_vertices(_ring(48, TPC1_SENSOR_R, z, cx, cy))
            mb.add_triangles(_fan(ci, ring), [0, 0, inward], LX, LX, surface=1, sensor=sid,
                             solid="sensors_top" if inward < 0 else "sensors_bottom")
            sid += 1
    surfaces = [Surface(r_diffuse=ptfe_r, p_absorb=1.0 - ptfe_r, grad_param=GRAD_REFLECTIVITY),
                Surface(p_detect=qe, p_absorb=1.0 - qe, flags=SURF_DETECT_FRONT_ONLY)]
    if plane:
        ring = mb.add_vertices(_ring(nseg, TPC1_R, TPC1_PLANE_Z))
        ci = mb.add_vertices([[0.0, 0.0, TPC1_PLANE_Z]])[0]
        mb.add_triangles(_fan(ci, ring), [0, 0, 1.0], LX, LX, surface=2, solid="plane")
        surfaces.append(Surface(p_transmit=plane_t, p_absorb=1.0 - plane_t,
                                grad_param=GRAD_TRANSPARENCY))
    return mb.build([lxe], surfaces, n_sensors=sid, name="tpc1+plane" if plane else "tpc1")


# ----------------------------------------------------------------------------
# DARWIN-scale TPC (G-darwin)
# ----------------------------------------------------------------------------

DARWIN_R_WALL = 1.30
DARWIN_Z_GATE = 0.0
DARWIN_Z_CATHODE = -2.598
DARWIN_Z_BSCREEN = -2.678
DARWIN_Z_IFACE = 0.002
DARWIN_TOP_FRONT = 0.007       # top windows: 5 mm above the liquid surface
DARWIN_BOT_FRONT = -2.688      # bottom windows: photocathode at -2.693 behind 5 mm quartz
DARWIN_WINDOW_T = 0.005
DARWIN_Z_TOPCAP = 0.020
DARWIN_Z_BOTCAP = -2.700
DARWIN_WINDOW_R = 0.0381
DARWIN_CATHODE_R = 0.032
DARWIN_PITCH = 0.080
DARWIN_STRIP_RMAX = 1.295
DARWIN_SEG_MAX = 0.04
DARWIN_SRC_R = 1.299
DARWIN_SRC_ZLO = -2.597
DARWIN_SRC_ZHI = -0.001


def darwin(n_wall: int = 256, sensor_pitch: float = DARWIN_PITCH, seg_max: float = DARWIN_SEG_MAX,
           electrodes: bool = True, coating: Optional[str] = None, single_phase: bool = False,
           bottom_array: bool = True, side_array: Optional[str] = None,
           fsr: Optional[str] = "copper", plates: str = "absorbing") -> Mesh:
    """DARWIN-shaped dual-phase TPC (about 4.8e5 triangles) and the paper's
    design variants (section "Alternative designs"):
      coating      "gate" or "all": electrodes covered with Al/MgF2 (90 %
                   reflective, 85 % of it specular);
      single_phase LXe up to the top array: no LXe/GXe interface, the gas
                   wall and top cap become liquid PTFE;
      bottom_array False: no bottom PMTs, the bottom PTFE reflector (0.99)
                   in their place;
      side_array   "pmt2" (2-inch square PMTs, 6 x 45 per plate) or "sipm"
                   (quad SiPMs, 22 x 165 per plate) on 24 absorbing backing
                   plates behind field-shaping rings instead of the liquid
                   PTFE wall (the 4-pi design);
      fsr          field-shaping rings of the 4-pi design: "copper" (45 %,
                   specular / diffuse 3.5), "coated" (Al/MgF2, 90 %, 17) or None;
      plates       backing plates of the 4-pi design: "absorbing" (the paper's
                   final choice) or "silicon" (reflectance from n = 0.81,
                   k = 1.86, the other option the paper tried).
    Sensor ids: top array, then bottom array, then the side array."""
    mb = MeshBuilder()
    LX, GX, QZ = 0, 1, 2
    S_PTFE_L, S_PTFE_G, S_SS, S_PC, S_CAP, S_COAT, S_CU, S_SIPM, S_SI = 0, 1, 2, 3, 4, 5, 6, 7, 8
    surfaces = [reflector(0.99, 0.05, grad_param=GRAD_REFLECTIVITY),
                reflector(0.80, 0.05),
                Surface(r_specular=0.20, r_diffuse=0.10, p_absorb=0.70),
                Surface(p_detect=1.0, flags=SURF_DETECT_FRONT_ONLY),
                Surface(p_absorb=1.0),
                reflector(0.90, 17.0),
                reflector(0.45, 3.5),
                Surface(r_specular=0.25, p_detect=0.75, flags=SURF_DETECT_FRONT_ONLY),
                complex_surface(SILICON_N, SILICON_K)]
    GAS = LX if single_phase else GX
    S_GAS_WALL = S_PTFE_L if single_phase else S_PTFE_G
    # side wall: 16 bands in the liquid (left out by the 4-pi design), one band in the gas
    z_liq = np.linspace(DARWIN_Z_BOTCAP, DARWIN_Z_IFACE, 17)
    zs = list(z_liq) + [DARWIN_Z_TOPCAP]
    rings = [mb.add_vertices(_ring(n_wall, DARWIN_R_WALL, z)) for z in zs]
    v = mb._vertex_array()
    for b in range(len(zs) - 1):
        tri = _band(rings[b], rings[b + 1])
        c = v[tri].mean(axis=1)
        gas = zs[b] >= DARWIN_Z_IFACE - 1e-12
        if side_array and not gas:
            continue
        mb.add_triangles(tri, c * np.array([1, 1, 0]), GAS if gas else LX, GAS if gas else LX,
                         surface=S_GAS_WALL if gas else S_PTFE_L,
                         solid="wall_gas" if gas else "wall_liquid")
    # end caps
    ci = mb.add_vertices([[0, 0, DARWIN_Z_BOTCAP]])[0]
    mb.add_triangles(_fan(ci, rings[0]), [0, 0, -1], LX, LX, surface=S_PTFE_L, solid="cap_bottom")
    ci = mb.add_vertices([[0, 0, DARWIN_Z_TOPCAP]])[0]
    mb.add_triangles(_fan(ci, rings[-1]), [0, 0, 1], GAS, GAS, surface=S_GAS_WALL, solid="cap_top")
    # liquid/gas interface, sharing the wall ring at the surface height
    iface_ring = rings[len(z_liq) - 1]
    if not single_phase:
        ci = mb.add_vertices([[0, 0, DARWIN_Z_IFACE]])[0]
        mb.add_triangles(_fan(ci, iface_ring), [0, 0, 1], LX, GX, surface=-1, solid="interface")
    # sensors: quartz window, photocathode on its back face, absorbing annulus and side
    centres = hex_centres(sensor_pitch, DARWIN_STRIP_RMAX - DARWIN_WINDOW_R)
    sid = 0
    arrays = [(DARWIN_TOP_FRONT, -1.0, GAS, "top")]
    if bottom_array:
        arrays.append((DARWIN_BOT_FRONT, 1.0, LX, "bottom"))
    for front, toward, xe, tag in arrays:
        tv, tt, ttags = _sensor_template(front, toward, xe, QZ, S_CAP, S_PC)
        nt_s = len(tt)
        for part in ("window_", "pmt_cap_", "photocathode_"):
            if part + tag not in mb.solid_names:
                mb.solid_names.append(part + tag)
        names = [mb.solid_names.index(x + tag) for x in ("window_", "pmt_cap_", "photocathode_")]
        k = len(centres)
        off = np.concatenate([centres, np.zeros((k, 1))], 1)
        verts = (tv[None, :, :] + off[:, None, :]).reshape(-1, 3)
        base = mb.add_vertices(verts)[0]
        tris = (tt[None, :, :] + base + len(tv) * np.arange(k)[:, None, None]).reshape(-1, 3)
        tags = np.tile(ttags, (k, 1))
        sensor_ids = sid + np.repeat(np.arange(k), nt_s)
        tags[:, 3] = np.where(tags[:, 2] == S_PC, sensor_ids, -1)
        tags[:, 4] = np.array(names)[tags[:, 4]]
        mb._t.append(tris.astype(np.int64))
        mb._tags.append(tags.astype(np.int64))
        sid += k
    # electrodes: zero-thickness two-sided stainless-steel strips (10 % of the pitch wide)
    if electrodes:
        for ze, pitch, tag in ((DARWIN_Z_GATE, 0.005, "gate"),
                               (DARWIN_Z_CATHODE, 0.0075, "cathode"),
                               (DARWIN_Z_BSCREEN, 0.0075, "bottom_screen")):
            coated = coating == "all" or (coating == "gate" and tag == "gate")
            _strips(mb, ze, pitch, 0.1 * pitch, DARWIN_STRIP_RMAX, seg_max, LX,
                    S_COAT if coated else S_SS, tag)
    if side_array:
        sid = _side_array(mb, n_wall, rings[0], iface_ring, side_array, fsr, sid, LX, QZ,
                          S_CAP, S_PC, S_SIPM, {"copper": S_CU, "coated": S_COAT}.get(fsr),
                          S_SI if plates == "silicon" else S_CAP)
    mats = [LXE, GXE, QUARTZ]
    name = "darwin" + "".join(f"+{k}" for k, on in (
        (f"coat-{coating}", coating), ("single-phase", single_phase),
        ("no-bottom", not bottom_array), (f"4pi-{side_array}-fsr-{fsr}", side_array),
        ("si-plates", side_array and plates == "silicon")) if on)
    return mb.build(mats, surfaces, n_sensors=sid, name=name)


def darwin_array_channels(mesh: Mesh) -> np.ndarray:
    """Channel of every sensor of a DARWIN mesh: 0 top array, 1 bottom array,
    2 side array (the paper's top / bottom / side LCE split)."""
    ch = np.full(mesh.n_sensors, -1, dtype=np.int32)
    names = mesh.solid_names
    for solid, c in (("photocathode_top", 0), ("photocathode_bottom", 1),
                     ("side_photocathode", 2), ("side_sipm", 2)):
        if solid in names:
            sel = (mesh.solid == names.index(solid)) & (mesh.sensor >= 0)
            ch[mesh.sensor[sel]] = c
    assert np.all(ch >= 0), "sensor without an array"
    return ch


# 4-pi design (section "4pi design"): field-shaping rings (FSRs) in the liquid,
# 24 flat backing plates behind them carrying the side photosensors
FSR_COUNT, FSR_STEP, FSR_HEIGHT, FSR_WIDTH = 92, 0.028, 0.020, 0.005
SIDE_PLATES = 24
SIDE_GAP_TO_ACTIVE = 0.0186       # FSR outer face to the sensors' active surface
PMT2_BODY, PMT2_ACTIVE, PMT2_WINDOW_T, PMT2_GRID = 0.056, 0.0485, 0.0025, (6, 45)
SIPM_HOLDER, SIPM_CELL, SIPM_GRID = 0.015, (0.00585, 0.00595), (22, 165)
SENSOR_SPACING = 0.0005
SIDE_OUTER_R = 1.340              # absorbing outer closure of the liquid annulus


def _quads(mb, corners, outward, mat_in, mat_out, surface, sensor, solid):
    """Add N planar quads (corners (N, 4, 3) in order around each) as two
    triangles each, oriented toward ``outward`` (N, 3)."""
    n = len(corners)
    base = mb.add_vertices(corners.reshape(-1, 3))[0]
    q = base + 4 * np.arange(n)[:, None] + np.arange(4)[None, :]
    tri = np.concatenate([q[:, [0, 1, 2]], q[:, [0, 2, 3]]], 0)
    out = np.concatenate([outward, outward], 0)
    sens = np.asarray(sensor)
    if sens.ndim:
        sens = np.concatenate([sens, sens], 0)
    mb.add_triangles(tri, out, mat_in, mat_out, surface=surface, sensor=sens, solid=solid)


def _rects(centre, u, w, half_u, half_w):
    """Corners (N, 4, 3) of rectangles centred at ``centre`` (N, 3) spanned by
    unit vectors u, w (N, 3) with half sizes half_u, half_w."""
    hu = half_u * u
    hw = half_w * w
    return np.stack([centre - hu - hw, centre + hu - hw, centre + hu + hw, centre - hu + hw], 1)


def _side_array(mb, n_wall, bottom_ring, top_ring, kind, fsr, sid, LX, QZ, S_ABS, S_PC, S_SIPM,
                S_FSR, S_PLATE):
    z_lo, z_hi = DARWIN_Z_BOTCAP, DARWIN_Z_IFACE
    z_mid = 0.5 * (z_lo + z_hi)
    r_in = DARWIN_R_WALL
    # field-shaping rings: rectangular-section rings r_in .. r_in + width
    if S_FSR is not None:
        for k in range(FSR_COUNT):
            zc = z_mid + (k - 0.5 * (FSR_COUNT - 1)) * FSR_STEP
            za, zb = zc - 0.5 * FSR_HEIGHT, zc + 0.5 * FSR_HEIGHT
            r0 = mb.add_vertices(_ring(n_wall, r_in, za))
            r1 = mb.add_vertices(_ring(n_wall, r_in, zb))
            r2 = mb.add_vertices(_ring(n_wall, r_in + FSR_WIDTH, za))
            r3 = mb.add_vertices(_ring(n_wall, r_in + FSR_WIDTH, zb))
            v = mb._vertex_array()
            for tri, outward in ((_band(r0, r1), -1.0), (_band(r2, r3), 1.0)):
                c = v[tri].mean(axis=1) * np.array([1, 1, 0])
                mb.add_triangles(tri, outward * c, LX, LX, surface=S_FSR, solid="fsr")
            mb.add_triangles(_annulus(r1, r3), [0, 0, 1], LX, LX, surface=S_FSR, solid="fsr")
            mb.add_triangles(_annulus(r0, r2), [0, 0, -1], LX, LX, surface=S_FSR, solid="fsr")
    # outer closure of the liquid annulus r_in .. SIDE_OUTER_R (absorbing)
    ob = mb.add_vertices(_ring(n_wall, SIDE_OUTER_R, z_lo))
    ot = mb.add_vertices(_ring(n_wall, SIDE_OUTER_R, z_hi))
    v = mb._vertex_array()
    tri = _band(ob, ot)
    mb.add_triangles(tri, v[tri].mean(axis=1) * np.array([1, 1, 0]), LX, LX, surface=S_ABS,
                     solid="side_closure")
    mb.add_triangles(_annulus(bottom_ring, ob), [0, 0, -1], LX, LX, surface=S_ABS,
                     solid="side_closure")
    mb.add_triangles(_annulus(top_ring, ot), [0, 0, 1], LX, LX, surface=S_ABS,
                     solid="side_closure")
    # backing plates: a 24-gon prism 1 mm behind the active surfaces (absorbing)
    a_active = r_in + FSR_WIDTH + SIDE_GAP_TO_ACTIVE
    a_plate = a_active + 0.001
    ang = 2 * np.pi * np.arange(SIDE_PLATES) / SIDE_PLATES
    nrm = np.stack([np.cos(ang), np.sin(ang), np.zeros_like(ang)], 1)
    tan = np.stack([-np.sin(ang), np.cos(ang), np.zeros_like(ang)], 1)
    zax = np.broadcast_to([0.0, 0.0, 1.0], nrm.shape)
    half_side = a_plate * math.tan(math.pi / SIDE_PLATES)
    pc = a_plate * nrm + np.array([0, 0, z_mid])
    _quads(mb, _rects(pc, tan, zax, half_side, 0.5 * (z_hi - z_lo)), -nrm, LX, LX, S_PLATE, -1,
           "backing_plate")
    # sensors on each plate, centred; u along the plate, w along z
    if kind == "pmt2":
        pitch, (nu, nw) = PMT2_BODY + SENSOR_SPACING, PMT2_GRID
    else:
        pitch, (nu, nw) = SIPM_HOLDER + SENSOR_SPACING, SIPM_GRID
    iu = (np.arange(nu) - 0.5 * (nu - 1)) * pitch
    iw = (np.arange(nw) - 0.5 * (nw - 1)) * pitch
    P, U, Wz = np.meshgrid(np.arange(SIDE_PLATES), iu, iw, indexing="ij")
    P, U, Wz = P.ravel(), U.ravel(), Wz.ravel()
    n_s = len(P)
    n_, t_, z_ = nrm[P], tan[P], np.broadcast_to([0.0, 0.0, 1.0], (n_s, 3))
    sensors = sid + np.arange(n_s)
    toward = -n_  # the sensors face the axis
    if kind == "pmt2":
        c_act = a_active * n_ + U[:, None] * t_ + (z_mid + Wz)[:, None] * z_
        ha, hb = 0.5 * PMT2_ACTIVE, 0.5 * PMT2_BODY
        c_win = c_act - PMT2_WINDOW_T * n_
        # photocathode on the back of the window: front (outer) side is the quartz
        _quads(mb, _rects(c_act, t_, z_, ha, ha), toward, LX, QZ, S_PC, sensors, "side_photocathode")
        # window front: a dielectric boundary, quartz inside
        _quads(mb, _rects(c_win, t_, z_, ha, ha), toward, QZ, LX, -1, -1, "side_window")
        # window sides: absorbing body
        for e_dir, e_oth in ((t_, z_), (-t_, z_), (z_, t_), (-z_, t_)):
            mid = 0.5 * (c_act + c_win) + ha * e_dir
            _quads(mb, _rects(mid, e_oth, n_, ha, 0.5 * PMT2_WINDOW_T), e_dir, QZ, LX, S_ABS, -1,
                   "side_body")
        # body frame around the active area, in the plane of the photocathode
        for e_dir, e_oth in ((t_, z_), (-t_, z_)):
            mid = c_act + 0.5 * (ha + hb) * e_dir
            _quads(mb, _rects(mid, e_dir, e_oth, 0.5 * (hb - ha), hb), toward, LX, LX, S_ABS, -1,
                   "side_body")
        for e_dir in (z_, -z_):
            mid = c_act + 0.5 * (ha + hb) * e_dir
            _quads(mb, _rects(mid, t_, e_dir, ha, 0.5 * (hb - ha)), toward, LX, LX, S_ABS, -1,
                   "side_body")
    else:
        c_h = a_active * n_ + U[:, None] * t_ + (z_mid + Wz)[:, None] * z_
        # ceramic holder 0.1 mm behind the cells (absorbing)
        _quads(mb, _rects(c_h + 0.0001 * n_, t_, z_, 0.5 * SIPM_HOLDER, 0.5 * SIPM_HOLDER), toward,
               LX, LX, S_ABS, -1, "side_holder")
        # four cells per quad SiPM, 2 x 2 around the holder centre; the film in
        # front of each reflects 25 % specularly, the rest reaches the active area
        du, dw = 0.5 * SIPM_CELL[0] + 0.0002, 0.5 * SIPM_CELL[1] + 0.0002
        cells = []
        for su in (-1.0, 1.0):
            for sw in (-1.0, 1.0):
                cells.append(_rects(c_h + su * du * t_ + sw * dw * z_, t_, z_,
                                    0.5 * SIPM_CELL[0], 0.5 * SIPM_CELL[1]))
        corners = np.concatenate(cells, 0)
        _quads(mb, corners, np.concatenate([toward] * 4, 0), LX, LX, S_SIPM,
               np.concatenate([sensors] * 4, 0), "side_sipm")
    return sid + n_s


def _sensor_template(front, toward, xe, qz, s_cap, s_pc, nw=32):
    """One 3-inch sensor centred on the z axis: vertices, oriented triangles and
    tags (mat_in, mat_out, surface, sensor placeholder, part index 0 window /
    1 cap / 2 photocathode)."""
    t = MeshBuilder()
    back = front - toward * DARWIN_WINDOW_T
    fc = t.add_vertices([[0, 0, front]])[0]
    fr = t.add_vertices(_ring(nw, DARWIN_WINDOW_R, front))
    br = t.add_vertices(_ring(nw, DARWIN_WINDOW_R, back))
    bc = t.add_vertices([[0, 0, back]])[0]
    pr = t.add_vertices(_ring(nw, DARWIN_CATHODE_R, back))
    # front face: xenon (outer) / quartz (inner), a dielectric boundary
    t.add_triangles(_fan(fc, fr), [0, 0, toward], qz, xe, surface=-1, solid="w")
    # side of the window: absorbing cap, normal pointing radially out of the quartz
    tri = _band(fr, br)
    c = t._vertex_array()[tri].mean(axis=1)
    t.add_triangles(tri, c * np.array([1, 1, 0]), qz, xe, surface=s_cap, solid="c")
    # photocathode on the back face; its normal points into the quartz (outer = quartz)
    t.add_triangles(_fan(bc, pr), [0, 0, toward], xe, qz, surface=s_pc, solid="p")
    t.add_triangles(_annulus(pr, br), [0, 0, toward], xe, qz, surface=s_cap, solid="c")
    part = {"w": 0, "c": 1, "p": 2}
    tags = np.concatenate(t._tags)
    tags[:, 4] = [part[t.solid_names[i]] for i in tags[:, 4]]
    return t._vertex_array(), np.concatenate(t._t), tags


def _strips(mb, ze, pitch, width, rmax, seg_max, medium, surf, tag):
    nmax = int(rmax / pitch) + 1
    ys = (np.arange(-nmax, nmax + 1)) * pitch
    quads = []
    allv = []
    base = mb._nv
    count = 0
    for y in ys:
        yo = abs(y) + 0.5 * width
        if yo >= rmax:
            continue
        half = math.sqrt(rmax * rmax - yo * yo)
        nseg = max(1, int(math.ceil(2 * half / seg_max)))
        xs = np.linspace(-half, half, nseg + 1)
        lo = np.stack([xs, np.full_like(xs, y - 0.5 * width), np.full_like(xs, ze)], 1)
        hi = np.stack([xs, np.full_like(xs, y + 0.5 * width), np.full_like(xs, ze)], 1)
        i_lo = base + count + np.arange(nseg + 1)
        i_hi = i_lo + nseg + 1
        allv.append(lo)
        allv.append(hi)
        count += 2 * (nseg + 1)
        a0, a1, b0, b1 = i_lo[:-1], i_lo[1:], i_hi[:-1], i_hi[1:]
        quads.append(np.concatenate([np.stack([a0, a1, b1], 1), np.stack([a0, b1, b0], 1)], 0))
    mb.add_vertices(np.concatenate(allv, 0))
    mb.add_triangles(np.concatenate(quads, 0), [0, 0, 1], medium, medium, surface=surf,
                     solid="electrode_" + tag)


# ----------------------------------------------------------------------------
# unit-test geometries
# ----------------------------------------------------------------------------

def icosphere(level: int):
    """Unit icosphere: vertices (float64) and outward-oriented faces."""
    t = (1.0 + 5 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t],
                  [0, -1, -t], [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]],
                 dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9],
                  [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2],
                  [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10],
                  [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}
        verts_l = list(verts)

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                p = (np.array(verts_l[a]) + np.array(verts_l[b])) * 0.5
                p /= np.linalg.norm(p)
                verts_l.append(tuple(p))
                cache[key] = len(verts_l) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        verts = verts_l
        f = np.array(nf, dtype=np.int64)
    return np.array(verts, dtype=np.float64), f


def sphere(radius=0.1, level=5, surface: Surface = None, lam_abs=INF, lam_ray=INF,
           inner_shell: Optional[Surface] = None, inner_level=4) -> Mesh:
    """Icosphere of the given radius filled with one medium; optional inner
    concentric icosphere at half the radius (a transparent shell)."""
    mb = MeshBuilder()
    v, f = icosphere(level)
    idx = mb.add_vertices(v * radius)
    cen = (v[f].mean(axis=1))
    mb.add_triangles(idx[f], cen, 0, 0, surface=0, sensor=0, solid="sphere")
    surfaces = [surface or Surface(p_detect=1.0)]
    if inner_shell is not None:
        v2, f2 = icosphere(inner_level)
        idx2 = mb.add_vertices(v2 * radius * 0.5)
        mb.add_triangles(idx2[f2], v2[f2].mean(axis=1), 0, 0, surface=1, solid="shell")
        surfaces.append(inner_shell)
    return mb.build([Material(1.69, lam_abs, lam_ray)], surfaces, n_sensors=1, name="sphere")


def box_faces(mb: MeshBuilder, lo, hi, mat_inner, mat_outer, surface, sensor=-1, solid="box",
              skip=()):
    """Axis-aligned box with outward normals, 2 triangles per face."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    c = np.array([[lo[0], lo[1], lo[2]], [hi[0], lo[1], lo[2]], [hi[0], hi[1], lo[2]],
                  [lo[0], hi[1], lo[2]], [lo[0], lo[1], hi[2]], [hi[0], lo[1], hi[2]],
                  [hi[0], hi[1], hi[2]], [lo[0], hi[1], hi[2]]])
    idx = mb.add_vertices(c)
    faces = {"-z": ([0, 1, 2, 3], [0, 0, -1]), "+z": ([4, 5, 6, 7], [0, 0, 1]),
             "-y": ([0, 1, 5, 4], [0, -1, 0]), "+y": ([3, 2, 6, 7], [0, 1, 0]),
             "-x": ([0, 3, 7, 4], [-1, 0, 0]), "+x": ([1, 2, 6, 5], [1, 0, 0])}
    for name, (q, nrm) in faces.items():
        if name in skip:
            continue
        q = idx[q]
        tri = np.array([[q[0], q[1], q[2]], [q[0], q[2], q[3]]])
        mb.add_triangles(tri, nrm, mat_inner, mat_outer, surface=surface, sensor=sensor,
                         solid=solid)
    return idx


SLAB_Z_BOTTOM = -0.10
SLAB_Z_IFACE = 0.0
SLAB_GAP = 0.067
SLAB_QUARTZ_T = 0.005


def slab() -> Mesh:
    """1 m x 1 m stack: detecting floor, LXe, LXe/GXe interface, 67 mm of GXe,
    a 5 mm quartz slab whose back face detects.  No bulk processes.
    Sensor 0 = the top (behind the quartz), sensor 1 = the floor."""
    mb = MeshBuilder()
    LX, GX, QZ = 0, 1, 2
    h = 0.5
    zq0 = SLAB_Z_IFACE + SLAB_GAP
    zq1 = zq0 + SLAB_QUARTZ_T
    levels = [SLAB_Z_BOTTOM, SLAB_Z_IFACE, zq0, zq1]
    corners = [mb.add_vertices([[-h, -h, z], [h, -h, z], [h, h, z], [-h, h, z]]) for z in levels]
    S_DET, S_ABS = 0, 1

    def quad(q, nrm, mi, mo, surf, sensor=-1, solid=""):
        tri = np.array([[q[0], q[1], q[2]], [q[0], q[2], q[3]]])
        mb.add_triangles(tri, nrm, mi, mo, surface=surf, sensor=sensor, solid=solid)

    quad(corners[0], [0, 0, -1], LX, LX, S_DET, sensor=1, solid="floor")
    quad(corners[1], [0, 0, 1], LX, GX, -1, solid="interface")
    quad(corners[2], [0, 0, 1], GX, QZ, -1, solid="quartz_front")
    quad(corners[3], [0, 0, -1], LX, QZ, S_DET, sensor=0, solid="quartz_back")
    for layer, med in ((0, LX), (1, GX), (2, QZ)):
        a, b = corners[layer], corners[layer + 1]
        for k in range(4):
            q = [a[k], a[(k + 1) % 4], b[(k + 1) % 4], b[k]]
            mid = (mb._vertex_array()[q]).mean(axis=0)
            quad(q, mid * np.array([1, 1, 0]), med, med, S_ABS, solid="side")
    mats = [Material(1.69, INF, INF), Material(1.00, INF, INF), Material(1.60, INF, INF)]
    return mb.build(mats, [Surface(p_detect=1.0), Surface(p_absorb=1.0)], n_sensors=2,
                    name="slab")


def disk_box(disk_radius=0.0381, distance=0.1, nseg=48) -> Mesh:
    """Absorbing 1 m cube centred on the origin with one detecting polygonal
    disk facing the origin at z = +distance."""
    mb = MeshBuilder()
    box_faces(mb, [-0.5] * 3, [0.5] * 3, 0, 0, surface=1, solid="box")
    ci = mb.add_vertices([[0, 0, distance]])[0]
    ring = mb.add_vertices(_ring(nseg, disk_radius, distance))
    mb.add_triangles(_fan(ci, ring), [0, 0, -1], 0, 0, surface=0, sensor=0, solid="disk")
    return mb.build([Material(1.69, INF, INF)], [Surface(p_detect=1.0), Surface(p_absorb=1.0)],
                    n_sensors=1, name="disk")


# ----------------------------------------------------------------------------
# sources (seeded; numpy's PCG64 for input positions and counts only)
# ----------------------------------------------------------------------------

SRC_POINTS = 0
SRC_UNIFORM_CYLINDER = 1
SRC_EXPLICIT = 2


@dataclasses.dataclass
class Sources:
    kind: int
    n_photons: int
    medium: int = 0
    positions: Optional[np.ndarray] = None     # float32 (n_src, 3) or (n_photons, 3)
    offsets: Optional[np.ndarray] = None       # int64 (n_src + 1,)
    count_per_source: int = 0
    per_source_events: bool = False
    directions: Optional[np.ndarray] = None    # EXPLICIT: float32 (n, 3)
    polarizations: Optional[np.ndarray] = None
    cyl_radius: float = 0.0
    cyl_zlo: float = 0.0
    cyl_zhi: float = 0.0
    time_profile: int = 0                      # 0: t = 0; 1: scintillation decay
    tau_singlet_ns: float = 0.0
    tau_triplet_ns: float = 0.0
    singlet_fraction: float = 0.0
    wavelength_nm: float = 174.8               # mean of the emission spectrum
    wavelength_fwhm_nm: float = 0.0            # 0: every photon at the mean

    @property
    def n_sources(self) -> int:
        if self.kind == SRC_POINTS:
            return int(self.positions.shape[0])
        return 0

    @property
    def n_events(self) -> int:
        return self.n_sources if (self.kind == SRC_POINTS and self.per_source_events) else 1


# scintillation time profile of LXe (section "Optical properties", table
# tab:optical): singlet / triplet time constants and the singlet fractions of
# nuclear-recoil (NR) and electronic-recoil (ER) events
SCINT_TAU_SINGLET_NS = 3.5
SCINT_TAU_TRIPLET_NS = 24.0
SINGLET_FRACTION_NR = 0.66
SINGLET_FRACTION_ER = 0.22


def with_scintillation(src: Sources, singlet_fraction=SINGLET_FRACTION_NR,
                       tau_singlet_ns=SCINT_TAU_SINGLET_NS,
                       tau_triplet_ns=SCINT_TAU_TRIPLET_NS) -> Sources:
    """The same sources with emission times from the two-exponential decay."""
    return dataclasses.replace(src, time_profile=1, tau_singlet_ns=float(tau_singlet_ns),
                               tau_triplet_ns=float(tau_triplet_ns),
                               singlet_fraction=float(singlet_fraction))


# components of the photon-loss table (section "Sources of photon losses",
# table tab:graveyard) in terms of the solids of the DARWIN-scale mesh
DARWIN_LOSS_COMPONENTS = {
    "PTFE reflectors": ("wall_liquid", "wall_gas"),
    "array caps": ("cap_top", "cap_bottom"),
    "LXe/GXe interface": ("interface",),
    "top PMTs": ("window_top", "pmt_cap_top", "photocathode_top"),
    "bottom PMTs": ("window_bottom", "pmt_cap_bottom", "photocathode_bottom"),
    "gate": ("electrode_gate",),
    "cathode": ("electrode_cathode",),
    "bottom screen": ("electrode_bottom_screen",),
}
DARWIN_MATERIAL_NAMES = ("LXe", "GXe", "quartz")
DARWIN_LOSS_COMPONENTS_4PI = dict(
    [(k, v) for k, v in DARWIN_LOSS_COMPONENTS.items() if k != "PTFE reflectors"]
    + [("PTFE reflectors", ("wall_gas",)), ("FSRs", ("fsr",)),
       ("side sensors", ("side_window", "side_body", "side_photocathode", "side_holder",
                         "side_sipm")),
       ("backing plates", ("backing_plate", "side_closure"))])


def loss_components(mesh: Mesh, components=None):
    """Loss group of every triangle and the group names: the solids of the
    mesh merged into the named components (solids not listed keep a group of
    their own)."""
    components = DARWIN_LOSS_COMPONENTS if components is None else components
    names = list(components)
    of_solid = {}
    for g, (name, solids) in enumerate(components.items()):
        for sname in solids:
            if sname in mesh.solid_names:
                of_solid[mesh.solid_names.index(sname)] = g
    for sid, sname in enumerate(mesh.solid_names):
        if sid not in of_solid:
            of_solid[sid] = len(names)
            names.append(sname)
    lut = np.array([of_solid[i] for i in range(len(mesh.solid_names))], dtype=np.int32)
    return lut[mesh.solid], names


# LXe scintillation spectrum (section "Optical properties"): Gaussian, mean
# 174.8 nm, FWHM 10.2 nm
SCINT_WAVELENGTH_NM, SCINT_FWHM_NM = 174.8, 10.2


def with_spectrum(src: Sources, mean_nm=SCINT_WAVELENGTH_NM, fwhm_nm=SCINT_FWHM_NM) -> Sources:
    """The same sources with wavelengths drawn from the Gaussian spectrum."""
    return dataclasses.replace(src, wavelength_nm=float(mean_nm), wavelength_fwhm_nm=float(fwhm_nm))


def uniform_points_in_cylinder(n, r_max, z_lo, z_hi, seed):
    rng = np.random.default_rng(seed)
    u = rng.random((n, 3))
    r = r_max * np.sqrt(u[:, 0])
    ph = 2 * np.pi * u[:, 1]
    z = z_lo + (z_hi - z_lo) * u[:, 2]
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], 1).astype(np.float32)


def point_sources(positions, counts=None, count_per_source=0, per_source_events=False,
                  medium=0) -> Sources:
    positions = np.ascontiguousarray(positions, dtype=np.float32).reshape(-1, 3)
    if counts is not None:
        counts = np.asarray(counts, dtype=np.int64)
        offsets = np.zeros(len(counts) + 1, dtype=np.int64)
        np.cumsum(counts, out=offsets[1:])
        n = int(offsets[-1])
        return Sources(SRC_POINTS, n, medium, positions, offsets, 0, per_source_events)
    n = int(count_per_source) * len(positions)
    return Sources(SRC_POINTS, n, medium, positions, None, int(count_per_source),
                   per_source_events)


def lognormal_counts(n, median, sigma, lo, hi, seed):
    rng = np.random.default_rng(seed)
    c = np.exp(np.log(median) + sigma * rng.standard_normal(n))
    return np.clip(np.rint(c), lo, hi).astype(np.int64)


def equal_volume_cell_centroids(nr, nphi, nz, r_max, z_lo, z_hi):
    """Centroids of nr x nphi x nz cells equal in volume: uniform in R^2, phi, z."""
    r2 = np.linspace(0.0, r_max * r_max, nr + 1)
    # centroid radius of an annular sector: (2/3)(r1^3 - r0^3)/(r1^2 - r0^2) * sinc(dphi/2)
    r0, r1 = np.sqrt(r2[:-1]), np.sqrt(r2[1:])
    dphi = 2 * np.pi / nphi
    rc = (2.0 / 3.0) * (r1 ** 3 - r0 ** 3) / (r1 ** 2 - r0 ** 2) * np.sinc(dphi / 2 / np.pi)
    phc = (np.arange(nphi) + 0.5) * dphi
    zc = z_lo + (np.arange(nz) + 0.5) * (z_hi - z_lo) / nz
    R, P, Z = np.meshgrid(rc, phc, zc, indexing="ij")
    return np.stack([R * np.cos(P), R * np.sin(P), Z], -1).reshape(-1, 3).astype(np.float32)


def explicit_sources(pos, dirs, pols, medium=0) -> Sources:
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    return Sources(SRC_EXPLICIT, len(pos), medium, positions=pos,
                   directions=np.ascontiguousarray(dirs, dtype=np.float32).reshape(-1, 3),
                   polarizations=np.ascontiguousarray(pols, dtype=np.float32).reshape(-1, 3))


def random_perpendicular(dirs, seed):
    """Unit vectors perpendicular to each row of dirs (random azimuth)."""
    rng = np.random.default_rng(seed)
    d = np.asarray(dirs, dtype=np.float64)
    a = np.where(np.abs(d[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    b1 = np.cross(d, a)
    b1 /= np.linalg.norm(b1, axis=1, keepdims=True)
    b2 = np.cross(d, b1)
    ang = 2 * np.pi * rng.random(len(d))
    return (np.cos(ang)[:, None] * b1 + np.sin(ang)[:, None] * b2).astype(np.float32)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

TPC1_SRC_R = 0.099
TPC1_SRC_ZHALF = 0.098


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    sources: Sources
    seed: int = 0
    grad_material: int = 0
    description: str = ""


def small_tpc(n_points=10, photons_per_point=10_000, seed=0) -> Workload:
    """Small TPC: 1e5 photons from 10 uniform-random points (one event)."""
    pos = uniform_points_in_cylinder(n_points, TPC1_SRC_R, -TPC1_SRC_ZHALF, TPC1_SRC_ZHALF, seed)
    src = point_sources(pos, count_per_source=photons_per_point)
    return Workload("small_tpc", tpc1(), src, seed,
                    description=f"G-tpc1 (4,128 triangles), {n_points} points x {photons_per_point}")


def darwin_tpc(n_photons=100_000_000, seed=0, mesh: Optional[Mesh] = None) -> Workload:
    """DARWIN-scale TPC: photons each at its own uniform point of the active volume."""
    src = Sources(SRC_UNIFORM_CYLINDER, int(n_photons), 0, cyl_radius=DARWIN_SRC_R,
                  cyl_zlo=DARWIN_SRC_ZLO, cyl_zhi=DARWIN_SRC_ZHI)
    return Workload("darwin_tpc", mesh if mesh is not None else darwin(), src, seed,
                    description=f"G-darwin, {n_photons:.3g} photons uniform in the active volume")


def batched_s1(n_events=4096, seed=0, mesh: Optional[Mesh] = None) -> Workload:
    """4096 S1-like point sources with log-normal photon counts (median 3e3,
    sigma = ln(1e3)/6 so that 1e2..1e5 is +-3 sigma), one event per source."""
    pos = uniform_points_in_cylinder(n_events, TPC1_SRC_R, -TPC1_SRC_ZHALF, TPC1_SRC_ZHALF,
                                     seed + 1)
    counts = lognormal_counts(n_events, 3000.0, math.log(1e3) / 6.0, 100, 100_000, seed + 2)
    src = point_sources(pos, counts=counts, per_source_events=True)
    return Workload("batched_s1", mesh if mesh is not None else tpc1(), src, seed,
                    description=f"G-tpc1, {n_events} log-normal sources, {src.n_photons} photons")


def differentiable(n_points=10, photons_per_point=1_000_000, seed=0,
                   lam_abs=50.0, lam_ray=0.4, ptfe_r=0.95, plane_t=0.9) -> Workload:
    pos = uniform_points_in_cylinder(n_points, TPC1_SRC_R, -TPC1_SRC_ZHALF, TPC1_SRC_ZHALF, seed)
    src = point_sources(pos, count_per_source=photons_per_point)
    mesh = tpc1(plane=True, ptfe_r=ptfe_r, plane_t=plane_t,
                lxe=Material(1.69, lam_abs, lam_ray))
    return Workload("differentiable", mesh, src, seed,
                    description=f"G-tpc1+plane, {n_points} x {photons_per_point} photons")


def lce_map(n=64, photons_per_voxel=10_000, seed=0) -> Workload:
    pos = equal_volume_cell_centroids(n, n, n, TPC1_SRC_R, -TPC1_SRC_ZHALF, TPC1_SRC_ZHALF)
    src = point_sources(pos, count_per_source=photons_per_voxel, per_source_events=True)
    return Workload("lce_map", tpc1(plane=True), src, seed,
                    description=f"G-tpc1+plane, {n}^3 voxels x {photons_per_voxel} photons")


def tpc1_top_bottom_channels(mesh: Mesh) -> np.ndarray:
    """Sensor -> channel map folding G-tpc1's 38 sensors into {top, bottom}."""
    return np.array([0 if s < 19 else 1 for s in range(mesh.n_sensors)], dtype=np.int32)
