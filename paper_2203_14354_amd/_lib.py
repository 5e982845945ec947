"""ctypes declarations of the C ABI in ``include/xephot.h``.

Loading fails loudly when ``libxephot.so`` has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxephot.so")

XP_OK = 0
ERRORS = {-1: "XP_ERR_INVALID_ARG", -2: "XP_ERR_STATE", -3: "XP_ERR_MESH", -4: "XP_ERR_HIP",
          -5: "XP_ERR_OOM", -6: "XP_ERR_UNSUPPORTED"}

FLAG_DETECT, FLAG_SENSOR_ABSORB, FLAG_SURFACE_ABSORB, FLAG_BULK_ABSORB = 1, 2, 3, 4
FLAG_ESCAPED, FLAG_MAX_STEPS, FLAG_NAN_ABORT, FLAG_GEOMETRY_ERROR = 5, 6, 7, 0x100
SRC_POINTS, SRC_UNIFORM_CYLINDER, SRC_EXPLICIT = 0, 1, 2
TIME_ZERO, TIME_SCINTILLATION = 0, 1


class XpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Material(ctypes.Structure):
    _fields_ = [("n", ctypes.c_float), ("abs_length", ctypes.c_float),
                ("rayleigh_length", ctypes.c_float)]


class Surface(ctypes.Structure):
    _fields_ = [("p_detect", ctypes.c_float), ("p_absorb", ctypes.c_float),
                ("r_diffuse", ctypes.c_float), ("r_specular", ctypes.c_float),
                ("p_transmit", ctypes.c_float), ("grad_param", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("model", ctypes.c_int32), ("n_re", ctypes.c_float),
                ("n_im", ctypes.c_float), ("film_n", ctypes.c_float),
                ("film_thickness_nm", ctypes.c_float)]


class BvhOptions(ctypes.Structure):
    _fields_ = [("max_leaf_size", ctypes.c_int32), ("sah_bins", ctypes.c_int32),
                ("split_budget", ctypes.c_float)]


class BvhInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_triangles", ctypes.c_int64),
                ("depth", ctypes.c_int32), ("max_stack", ctypes.c_int32),
                ("node_bytes", ctypes.c_int64), ("triangle_bytes", ctypes.c_int64),
                ("build_seconds", ctypes.c_double), ("n_references", ctypes.c_int64)]


class Sources(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("medium", ctypes.c_int32),
                ("n_photons", ctypes.c_int64), ("n_sources", ctypes.c_int64),
                ("positions", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("count_per_source", ctypes.c_int64), ("per_source_events", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("directions", ctypes.c_void_p),
                ("polarizations", ctypes.c_void_p), ("cyl_radius", ctypes.c_float),
                ("cyl_zlo", ctypes.c_float), ("cyl_zhi", ctypes.c_float),
                ("time_profile", ctypes.c_int32), ("tau_singlet_ns", ctypes.c_float),
                ("tau_triplet_ns", ctypes.c_float), ("singlet_fraction", ctypes.c_float),
                ("wavelength_nm", ctypes.c_float), ("wavelength_fwhm_nm", ctypes.c_float)]


class ExtraTallies(ctypes.Structure):
    _fields_ = [("d_time_hist", ctypes.c_void_p), ("n_time_bins", ctypes.c_int32),
                ("time_bin_ns", ctypes.c_float), ("d_loss", ctypes.c_void_p)]


class RunParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("pid_base", ctypes.c_uint64),
                ("max_steps", ctypes.c_int32), ("eps", ctypes.c_float),
                ("grad_material", ctypes.c_int32), ("surface_offset", ctypes.c_float)]


class LaunchCfg(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("lds_levels", ctypes.c_int32),
                ("stack_lds", ctypes.c_int32), ("wave_batch", ctypes.c_int32),
                ("block_tally", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# the BVH as xp_bvh_build_host returns it: 128-byte nodes, 48-byte triangle records
NODE_DTYPE = np.dtype([("lo_x", np.float32, 4), ("hi_x", np.float32, 4), ("lo_y", np.float32, 4),
                       ("hi_y", np.float32, 4), ("lo_z", np.float32, 4), ("hi_z", np.float32, 4),
                       ("child", np.int32, 4), ("reserved", np.int32, 4)])
TRIREC_DTYPE = np.dtype([("v0", np.float32, 3), ("tri", np.int32), ("v1", np.float32, 3),
                         ("packed", np.int32), ("v2", np.float32, 3), ("sensor", np.int32)])
EMPTY_CHILD = -2 ** 31

RECORD_DTYPE = np.dtype([
    ("flag", np.int32), ("last_tri", np.int32), ("sensor", np.int32), ("steps", np.int32),
    ("event", np.int32), ("medium", np.int32), ("n_scatter", np.int32), ("reserved", np.int32),
    ("pos", np.float32, 3), ("time", np.float32), ("dir", np.float32, 3),
    ("path_len", np.float32), ("pol", np.float32, 3), ("sum_inv_r", np.float32),
    ("sum_inv_t", np.float32), ("wavelength", np.float32), ("pad", np.float32, 2)])
assert RECORD_DTYPE.itemsize == 96

# every symbol the header declares
EXPORTS = ["xp_context_create", "xp_context_destroy", "xp_last_error", "xp_load_mesh",
           "xp_set_materials", "xp_set_material_dispersion", "xp_set_surfaces",
           "xp_set_channel_map", "xp_build_bvh",
           "xp_bvh_stats", "xp_propagate", "xp_propagate_ex", "xp_propagate_static",
           "xp_set_loss_groups",
           "xp_time_quantile", "xp_backward", "xp_autotune", "xp_closest_hit", "xp_sample",
           "xp_sample_emission_time", "xp_sample_wavelength", "xp_surface_reflectance",
           "xp_stream_read", "xp_valu_probe",
           "xp_bvh_build_host", "xp_version"]

_lib = None


def load():
    """Load libxephot.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python -m paper_2203_14354_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, F = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                           ctypes.c_float)
    sig = {
        "xp_context_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(P)]),
        "xp_context_destroy": (None, [P]),
        "xp_last_error": (ctypes.c_char_p, [P]),
        "xp_load_mesh": (ctypes.c_int, [P, P, I64, P, I64, P, P, P, P]),
        "xp_set_materials": (ctypes.c_int, [P, P, I32]),
        "xp_set_material_dispersion": (ctypes.c_int, [P, I32, I32, P, P, P, P]),
        "xp_set_surfaces": (ctypes.c_int, [P, P, I32]),
        "xp_set_channel_map": (ctypes.c_int, [P, P, I32, I32]),
        "xp_build_bvh": (ctypes.c_int, [P, P]),
        "xp_bvh_stats": (ctypes.c_int, [P, P]),
        "xp_propagate": (ctypes.c_int, [P, P, P, P, P, P, P, P, P]),
        "xp_propagate_ex": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, P]),
        "xp_propagate_static": (ctypes.c_int, [P, P, P, P, P, P, P, P, P]),
        "xp_set_loss_groups": (ctypes.c_int, [P, P, I32]),
        "xp_time_quantile": (ctypes.c_int, [P, I64, I32, F, F, P, P]),
        "xp_backward": (ctypes.c_int, [P, P, P, P, P, P, P]),
        "xp_autotune": (ctypes.c_int, [P, P, P, I64, P, P]),
        "xp_closest_hit": (ctypes.c_int, [P, I64, P, P, P, F, F, I32, P, P, P]),
        "xp_sample": (ctypes.c_int, [I32, U64, U64, I64, P, P, F, F, F, P, P, P]),
        "xp_sample_emission_time": (ctypes.c_int, [U64, U64, I64, F, F, F, P, P, P]),
        "xp_sample_wavelength": (ctypes.c_int, [U64, U64, I64, F, F, P, P]),
        "xp_stream_read": (ctypes.c_int, [P, I64, I32, I32, P, P]),
        "xp_valu_probe": (ctypes.c_int, [I32, I32, I32, P, P]),
        "xp_surface_reflectance": (ctypes.c_int, [I32, F, F, F, F, F, F, I64, P, P, P, P]),
        "xp_bvh_build_host": (ctypes.c_int, [P, I64, P, I64, P, P, P, I64, P, I64]),
        "xp_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(rc, ctx=None):
    if rc != XP_OK:
        msg = load().xp_last_error(ctx)
        raise XpError(rc, msg.decode() if msg else "")
    return rc
