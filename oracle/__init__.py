"""CPU oracle for the photon transport -- TEST INFRASTRUCTURE ONLY.

A plain FP64 C++ implementation (``xeoracle.cpp``) of what the HIP path
computes, loaded with ctypes.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the library itself never
does.  It shares no code with the HIP path: both receive the same input arrays
built by ``paper_2203_14354_amd.workloads`` and compute independently.

The same source built with ``-DXEORACLE_FP32`` (``fp32=True`` below) computes
the transport in single precision: a diagnostic build that tells whether a
photon on which the HIP path and the FP64 oracle part is one where FP32
rounding alone changes the outcome.  Results of record are the FP64 build's.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xeoracle.cpp")
_LIB = os.path.join(_HERE, "libxeoracle.so")
_LIB32 = os.path.join(_HERE, "libxeoracle_fp32.so")

F_DETECT, F_SENSOR_ABSORB, F_SURFACE_ABSORB, F_BULK_ABSORB = 1, 2, 3, 4
F_ESCAPED, F_MAX_STEPS, F_NAN_ABORT, F_GEOMETRY_ERROR = 5, 6, 7, 0x100

RECORD_DTYPE = np.dtype([
    ("flag", np.int32), ("last_tri", np.int32), ("sensor", np.int32), ("steps", np.int32),
    ("event", np.int32), ("medium", np.int32), ("n_scatter", np.int32), ("pad", np.int32),
    ("pos", np.float64, 3), ("dir", np.float64, 3), ("pol", np.float64, 3),
    ("time", np.float64), ("path_len", np.float64), ("sum_inv_r", np.float64),
    ("sum_inv_t", np.float64), ("wavelength", np.float64),
])
assert RECORD_DTYPE.itemsize == 32 + 9 * 8 + 5 * 8


def _compile(out, defines):
    tmp = out + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           *defines, "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle (g++, OpenMP, no FMA contraction, portable -O2) and
    its FP32 diagnostic build."""
    for out, defines in ((_LIB, []), (_LIB32, ["-DXEORACLE_FP32"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            _compile(out, defines)
    return _LIB


_libs = {}


def lib(fp32: bool = False):
    """The FP64 oracle library (fp32=True: its FP32 diagnostic build)."""
    key = bool(fp32)
    if key not in _libs:
        path = _LIB32 if key else _LIB
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        P, I32, I64, U64, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                               ctypes.c_double)
        L.oracle_scene_create.restype = P
        L.oracle_scene_create.argtypes = [P, I64, P, I64, P, P, P, P, P, I32, P, P, P, I32, P,
                                          I32, I32, I32]
        L.oracle_scene_set_dispersion.argtypes = [P, I32, I32, P, P, P, P]
        L.oracle_scene_destroy.argtypes = [P]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_run.argtypes = [P, I32, I32, I64, I64, P, P, I64, I32, P, P, D, D, D, I32, D, D, D,
                                 D, D, U64, U64,
                                 I32, D, I32, D, I64, I64, P, P, P, I32]
        L.oracle_philox.argtypes = [P, P, P]
        L.oracle_u01.restype = D
        L.oracle_u01.argtypes = [ctypes.c_uint32]
        L.oracle_is_fp32.restype = I32
        L.oracle_sample.argtypes = [I32, U64, U64, I64, P, P, D, D, D, P, P]
        L.oracle_boundary.restype = I32
        L.oracle_boundary.argtypes = [I32, P, P, P, D, D, D, P, P]
        L.oracle_model_boundary.restype = I32
        L.oracle_model_boundary.argtypes = [I32, P, P, P, D, D, D, D, D, D, D, P, P]
        L.oracle_closest_hit.argtypes = [P, I64, P, P, D, D, P, I32, P, P]
        L.oracle_emission_time.argtypes = [U64, U64, I64, D, D, D, P, P]
        L.oracle_wavelength.argtypes = [U64, U64, I64, D, D, P]
        L.oracle_surface_reflectance.argtypes = [I32, D, D, D, D, D, D, I64, P, P, P]
        L.oracle_material_at.argtypes = [P, I32, I64, P, P]
        L.oracle_max_threads.restype = I32
        assert L.oracle_is_fp32() == (1 if key else 0)
        _libs[key] = L
    return _libs[key]


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Scene:
    """Oracle copy of a mesh plus its optical tables."""

    def __init__(self, mesh, channel_of_sensor=None, n_channels=None, use_bvh=False,
                 fp32=False):
        from paper_2203_14354_amd.workloads import materials_array, surfaces_array
        self.mesh = mesh
        self.lib = lib(fp32)
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        v = keep(mesh.vertices, np.float32)
        t = keep(mesh.triangles, np.int32)
        mi, mo = keep(mesh.mat_inner, np.int32), keep(mesh.mat_outer, np.int32)
        su, se = keep(mesh.surface, np.int32), keep(mesh.sensor, np.int32)
        mats = keep(materials_array(mesh.materials), np.float32)
        sp, stags, sopt = surfaces_array(mesh.surfaces)
        sp, stags, sopt = keep(sp, np.float32), keep(stags, np.int32), keep(sopt, np.float32)
        if channel_of_sensor is None:
            ch = keep(np.arange(mesh.n_sensors, dtype=np.int32), np.int32)
            nch = mesh.n_sensors
        else:
            ch = keep(channel_of_sensor, np.int32)
            nch = int(n_channels if n_channels is not None else ch.max() + 1)
        self.n_channels = nch
        self.handle = self.lib.oracle_scene_create(
            _p(v), len(v), _p(t), len(t), _p(mi), _p(mo), _p(su), _p(se), _p(mats), len(mats),
            _p(sp), _p(stags), _p(sopt), len(sp), _p(ch), mesh.n_sensors, nch,
            1 if use_bvh else 0)
        for m, mat in enumerate(mesh.materials):
            tab = getattr(mat, "dispersion", None)
            if tab is not None:
                tab = keep(np.asarray(tab, dtype=np.float32).reshape(-1, 4).T.copy(), np.float32)
                self.lib.oracle_scene_set_dispersion(self.handle, m, tab.shape[1], _p(tab[0]),
                                                  _p(tab[1]), _p(tab[2]), _p(tab[3]))

    def material_at(self, m, lambdas):
        """(index, absorption length, Rayleigh length) of material m at the
        given wavelengths (nm), from its dispersion table."""
        lam = np.ascontiguousarray(lambdas, dtype=np.float64).reshape(-1)
        out = np.zeros((len(lam), 3))
        self.lib.oracle_material_at(self.handle, int(m), len(lam), _p(lam), _p(out))
        return out

    def __del__(self):
        if getattr(self, "handle", None) and getattr(self, "lib", None) is not None:
            self.lib.oracle_scene_destroy(self.handle)
            self.handle = None

    def closest_hit(self, orig, dirs, tmin=0.0, tmax=np.inf, skip=None, brute=False):
        o = np.ascontiguousarray(orig, dtype=np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int32)
        tri = np.empty(len(o), dtype=np.int32)
        t = np.empty(len(o), dtype=np.float64)
        self.lib.oracle_closest_hit(self.handle, len(o), _p(o), _p(d), float(tmin), float(tmax),
                                 _p(sk), 1 if brute else 0, _p(tri), _p(t))
        return tri, t


SURFACE_OFFSET = 2e-6  # m


def run(scene: Scene, sources, seed=0, pid_base=0, max_steps=10_000, eps=0.0, grad_material=0,
        i_begin=0, i_end=None, records=True, hit_map=True, grad=False, n_threads=0,
        surface_offset=SURFACE_OFFSET):
    """Propagate launch-local photons [i_begin, i_end).  Returns a dict with
    'records' (RECORD_DTYPE array), 'hit_map' (int64 [events, channels]) and
    'grad' (float64 [events, channels, 4]) as requested."""
    s = sources
    if i_end is None:
        i_end = s.n_photons
    n = i_end - i_begin
    keep = []

    def arr(a, dt):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    pos = arr(s.positions, np.float32)
    offs = arr(s.offsets, np.int64)
    dirs = arr(s.directions, np.float32)
    pols = arr(s.polarizations, np.float32)
    out = {}
    rec = np.zeros(n, dtype=RECORD_DTYPE) if records else None
    hm = np.zeros((s.n_events, scene.n_channels), dtype=np.int64) if hit_map else None
    gr = np.zeros((s.n_events, scene.n_channels, 4), dtype=np.float64) if grad else None
    n_src = s.n_sources if s.kind == 0 else 0
    # the time-profile parameters enter as the FP32 values the library receives
    tp = int(getattr(s, "time_profile", 0))
    f32 = lambda x: float(np.float32(x))
    scene.lib.oracle_run(scene.handle, s.kind, s.medium, s.n_photons, n_src, _p(pos), _p(offs),
                     int(s.count_per_source), 1 if s.per_source_events else 0, _p(dirs), _p(pols),
                     float(s.cyl_radius), float(s.cyl_zlo), float(s.cyl_zhi), tp,
                     f32(getattr(s, "tau_singlet_ns", 0.0)), f32(getattr(s, "tau_triplet_ns", 0.0)),
                     f32(getattr(s, "singlet_fraction", 0.0)),
                     f32(getattr(s, "wavelength_nm", 0.0)), f32(getattr(s, "wavelength_fwhm_nm", 0.0)),
                     int(seed),
                     int(pid_base), int(max_steps), float(eps), int(grad_material),
                     float(surface_offset), int(i_begin),
                     int(i_end), _p(rec), _p(hm), _p(gr), int(n_threads))
    if records:
        out["records"] = rec
    if hit_map:
        out["hit_map"] = hm
    if grad:
        out["grad"] = gr
    return out


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox(_p(c), _p(k), _p(o))
    return o


def u01(x: int) -> float:
    return lib().oracle_u01(int(x))


def sample(kind, seed, pid0, n, in_dir=None, in_pol=None, cyl=(0.0, 0.0, 0.0), fp32=False):
    """kind 0 emission, 1 Lambertian about in_dir, 2 Rayleigh from (in_dir, in_pol),
    3 uniform-cylinder positions (returned in the first array)."""
    di = None if in_dir is None else np.ascontiguousarray(
        np.broadcast_to(np.asarray(in_dir, np.float64), (n, 3)))
    pi = None if in_pol is None else np.ascontiguousarray(
        np.broadcast_to(np.asarray(in_pol, np.float64), (n, 3)))
    od = np.zeros((n, 3))
    op = np.zeros((n, 3))
    lib(fp32).oracle_sample(int(kind), int(seed), int(pid0), int(n), _p(di), _p(pi), float(cyl[0]),
                        float(cyl[1]), float(cyl[2]), _p(od), _p(op))
    return od, op


def emission_time(seed, pid0, n, tau_singlet, tau_triplet, singlet_fraction):
    """Scintillation emission times (ns) and states (1 singlet) of photon ids
    pid0 .. pid0+n-1 (parameters taken as FP32 values, as the library does)."""
    t = np.zeros(n)
    st = np.zeros(n, dtype=np.int32)
    f32 = lambda x: float(np.float32(x))
    lib().oracle_emission_time(int(seed), int(pid0), int(n), f32(tau_singlet), f32(tau_triplet),
                               f32(singlet_fraction), _p(t), _p(st))
    return t, st


def wavelength(seed, pid0, n, mean, fwhm):
    """Emission wavelengths (nm) of photon ids pid0 .. pid0+n-1 (parameters as FP32)."""
    out = np.zeros(n)
    lib().oracle_wavelength(int(seed), int(pid0), int(n), float(np.float32(mean)),
                            float(np.float32(fwhm)), _p(out))
    return out


def surface_reflectance(model, n1, n_re, n_im, film_n=0.0, film_d_nm=0.0, lam=174.8, cos_i=1.0):
    """|r_s|^2 and |r_p|^2 of a complex-index (model 1) or thin-film (model 2)
    surface at the given incidence cosines."""
    c = np.ascontiguousarray(np.atleast_1d(cos_i), dtype=np.float64)
    rs, rp = np.zeros(len(c)), np.zeros(len(c))
    lib().oracle_surface_reflectance(int(model), float(n1), float(n_re), float(n_im), float(film_n),
                                     float(film_d_nm), float(lam), len(c), _p(c), _p(rs), _p(rp))
    return rs, rp


# ---- tallies over photon records, written out from their definitions ----

def time_histogram(records, n_events, n_bins, bin_ns, time_dtype=np.float64):
    """Detected photons per event by arrival-time bin: bin floor(t / bin_ns),
    the last bin open-ended (section "Light collection efficiency": t90 is
    taken from the arrival times of detected photons).  With time_dtype
    float32 the bin index is floor(t * inv) in FP32 with inv = fp32(1 / bin_ns)."""
    det = (records["flag"] & 0xFF) == F_DETECT
    t = records["time"][det]
    ev = records["event"][det].astype(np.int64)
    if time_dtype == np.float32:
        f = t.astype(np.float32) * np.float32(1.0 / bin_ns)
    else:
        f = t.astype(np.float64) / bin_ns
    b = np.where(f < n_bins - 1, np.floor(np.maximum(f, 0)), n_bins - 1).astype(np.int64)
    h = np.zeros((n_events, n_bins), dtype=np.int64)
    np.add.at(h, (ev, b), 1)
    return h


def time_quantile(hist, bin_ns, q=0.9):
    """Per event, the time by which a fraction q of the detected photons had
    arrived: the first bin where the cumulative count reaches q * total, with
    linear interpolation inside it (NaN: no photons; inf: the open last bin)."""
    hist = np.asarray(hist, dtype=np.int64)
    out = np.full(hist.shape[0], np.nan)
    for e in range(hist.shape[0]):
        h = hist[e]
        total = int(h.sum())
        if total == 0:
            continue
        target = q * total
        cum = 0
        for b in range(len(h)):
            c = int(h[b])
            if c > 0 and cum + c >= target:
                out[e] = np.inf if b == len(h) - 1 else (b + (target - cum) / c) * bin_ns
                break
            cum += c
    return out


def loss_table(records, tri_group, n_groups, n_materials):
    """Photons by where they ended (section "Sources of photon losses", table
    tab:graveyard): rows 0..n_groups-1 are triangle groups (photons ending on
    a surface: detected, absorbed in a sensor, absorbed on a surface), rows
    n_groups + m the materials (bulk absorption, escape, step limit, NaN);
    columns are the terminal flags."""
    fl = records["flag"] & 0xFF
    on_surface = (fl >= F_DETECT) & (fl <= F_SURFACE_ABSORB) & (records["last_tri"] >= 0)
    tg = np.asarray(tri_group, dtype=np.int64)
    row = np.where(on_surface, tg[np.maximum(records["last_tri"], 0)],
                   n_groups + records["medium"].astype(np.int64))
    t = np.zeros((n_groups + n_materials, 8), dtype=np.int64)
    np.add.at(t, (row, fl), 1)
    return t


def boundary(mode, d, e, n, n1=1.0, n2=1.0, u=0.5, fp32=False):
    """One boundary event (mode 0 Fresnel between indices n1 -> n2, mode 1
    specular) of a photon (direction d, polarization e) on a plane of unit
    normal n (either orientation).  Returns (transmitted, new direction, new
    polarization)."""
    d = np.ascontiguousarray(d, np.float64)
    e = np.ascontiguousarray(e, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    od, op = np.zeros(3), np.zeros(3)
    tr = lib(fp32).oracle_boundary(int(mode), _p(d), _p(e), _p(n), float(n1), float(n2), float(u),
                               _p(od), _p(op))
    return bool(tr), od, op


def model_boundary(model, d, e, n, n1, n_re, n_im, film_n=0.0, film_d_nm=0.0, lam=174.8, u=0.5,
                   fp32=False):
    """One reflection off a complex-index (model 1) or thin-film (model 2)
    surface: returns (reflected, new direction, new polarization); a photon
    that is not reflected keeps its direction and polarization."""
    d = np.ascontiguousarray(d, np.float64)
    e = np.ascontiguousarray(e, np.float64)
    n = np.ascontiguousarray(n, np.float64)
    od, op = d.copy(), e.copy()
    r = lib(fp32).oracle_model_boundary(int(model), _p(d), _p(e), _p(n), float(n1), float(n_re),
                                        float(n_im), float(film_n), float(film_d_nm), float(lam),
                                        float(u), _p(od), _p(op))
    return bool(r), od, op


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def is_fp32(fp32: bool = False) -> bool:
    return bool(lib(fp32).oracle_is_fp32())
