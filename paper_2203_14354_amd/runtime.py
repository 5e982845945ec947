"""Python front end of the transport library: argument marshalling only.

torch provides device memory and streams; every step of the transport runs in
the library's HIP kernels (``libxephot.so``), reached through the C ABI.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import (RECORD_DTYPE, BvhInfo, BvhOptions, ExtraTallies, LaunchCfg, Material,
                   RunParams, Sources, Surface, check, load)


SURFACE_OFFSET = 2e-6  # m, restart distance from a surface after an interaction


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _host_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def current_stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class DeviceSources:
    """A ``workloads.Sources`` with its arrays resident on the device."""

    def __init__(self, src, device):
        self.src = src
        self.device = device

        def up(a, dt):
            if a is None:
                return None
            return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)

        self.positions = up(src.positions, np.float32)
        self.offsets = up(src.offsets, np.int64)
        self.directions = up(src.directions, np.float32)
        self.polarizations = up(src.polarizations, np.float32)
        self.n_photons = int(src.n_photons)
        self.n_events = src.n_events

    def struct(self, n_photons: Optional[int] = None) -> Sources:
        s = self.src
        return Sources(kind=s.kind, medium=s.medium,
                       n_photons=self.n_photons if n_photons is None else int(n_photons),
                       n_sources=s.n_sources if s.kind == _lib.SRC_POINTS else 0,
                       positions=_ptr(self.positions), offsets=_ptr(self.offsets),
                       count_per_source=int(s.count_per_source),
                       per_source_events=1 if s.per_source_events else 0, reserved=0,
                       directions=_ptr(self.directions), polarizations=_ptr(self.polarizations),
                       cyl_radius=s.cyl_radius, cyl_zlo=s.cyl_zlo, cyl_zhi=s.cyl_zhi,
                       time_profile=int(getattr(s, "time_profile", 0)),
                       tau_singlet_ns=float(getattr(s, "tau_singlet_ns", 0.0)),
                       tau_triplet_ns=float(getattr(s, "tau_triplet_ns", 0.0)),
                       singlet_fraction=float(getattr(s, "singlet_fraction", 0.0)),
                       wavelength_nm=float(getattr(s, "wavelength_nm", 0.0)),
                       wavelength_fwhm_nm=float(getattr(s, "wavelength_fwhm_nm", 0.0)))


class Detector:
    """A mesh + optical tables + BVH resident on one GPU."""

    def __init__(self, mesh, device=0, channel_of_sensor=None, n_channels=None,
                 max_leaf_size=1, sah_bins=32, split_budget=0.0):
        self.lib = load()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.mesh = mesh
        ctx = ctypes.c_void_p()
        check(self.lib.xp_context_create(self.device.index or 0, ctypes.byref(ctx)))
        self.ctx = ctx
        self._upload_mesh(mesh)
        self.set_materials(mesh.materials)
        self.set_surfaces(mesh.surfaces)
        if channel_of_sensor is not None:
            ch = np.ascontiguousarray(channel_of_sensor, dtype=np.int32)
            nch = int(n_channels if n_channels is not None else ch.max() + 1)
            check(self.lib.xp_set_channel_map(self.ctx, _host_ptr(ch), len(ch), nch), self.ctx)
            self.n_channels = nch
        else:
            self.n_channels = int(max(mesh.n_sensors, int(mesh.sensor.max()) + 1, 1))
        check(self.lib.xp_build_bvh(self.ctx, ctypes.byref(
            BvhOptions(max_leaf_size, sah_bins, split_budget))), self.ctx)
        info = BvhInfo()
        check(self.lib.xp_bvh_stats(self.ctx, ctypes.byref(info)), self.ctx)
        self.bvh = {k: getattr(info, k) for k, _ in BvhInfo._fields_}

    def _upload_mesh(self, mesh):
        self._mesh_arrays = [np.ascontiguousarray(a, dtype=dt) for a, dt in (
            (mesh.vertices, np.float32), (mesh.triangles, np.int32), (mesh.mat_inner, np.int32),
            (mesh.mat_outer, np.int32), (mesh.surface, np.int32), (mesh.sensor, np.int32))]
        v, t, mi, mo, su, se = self._mesh_arrays
        check(self.lib.xp_load_mesh(self.ctx, _host_ptr(v), len(v), _host_ptr(t), len(t),
                                    _host_ptr(mi), _host_ptr(mo), _host_ptr(su), _host_ptr(se)),
              self.ctx)

    def set_materials(self, mats):
        arr = (Material * len(mats))(*[Material(m.n, m.abs_length, m.rayleigh_length)
                                       for m in mats])
        check(self.lib.xp_set_materials(self.ctx, arr, len(mats)), self.ctx)
        for i, m in enumerate(mats):
            tab = getattr(m, "dispersion", None)
            if tab is not None:
                t = np.ascontiguousarray(np.asarray(tab, dtype=np.float32).reshape(-1, 4).T)
                cols = [np.ascontiguousarray(c) for c in t]
                check(self.lib.xp_set_material_dispersion(
                    self.ctx, i, t.shape[1], *[_host_ptr(c) for c in cols]), self.ctx)
        self.materials = list(mats)

    def set_surfaces(self, surfs):
        arr = (Surface * len(surfs))(*[Surface(s.p_detect, s.p_absorb, s.r_diffuse, s.r_specular,
                                               s.p_transmit, s.grad_param, s.flags,
                                               getattr(s, "model", 0), getattr(s, "n_re", 0.0),
                                               getattr(s, "n_im", 0.0), getattr(s, "film_n", 0.0),
                                               getattr(s, "film_thickness_nm", 0.0))
                                       for s in surfs])
        check(self.lib.xp_set_surfaces(self.ctx, arr, len(surfs)), self.ctx)
        self.surfaces = list(surfs)

    def set_loss_groups(self, group_of_triangle, n_groups=None):
        """Loss group of every mesh triangle (e.g. the mesh's solid ids)."""
        g = np.ascontiguousarray(group_of_triangle, dtype=np.int32)
        ng = int(n_groups if n_groups is not None else g.max() + 1)
        check(self.lib.xp_set_loss_groups(self.ctx, _host_ptr(g), ng), self.ctx)
        self.n_groups = ng

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.xp_context_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def sources(self, src) -> DeviceSources:
        return src if isinstance(src, DeviceSources) else DeviceSources(src, self.device)

    @staticmethod
    def run_params(seed=0, pid_base=0, max_steps=10_000, eps=0.0, grad_material=0,
                   surface_offset=SURFACE_OFFSET) -> RunParams:
        return RunParams(seed=int(seed), pid_base=int(pid_base), max_steps=int(max_steps),
                         eps=float(eps), grad_material=int(grad_material),
                         surface_offset=float(surface_offset))

    def propagate(self, src, seed=0, pid_base=0, max_steps=10_000, eps=0.0, grad_material=0,
                  hit_map: Optional[torch.Tensor] = None, grad=False, records=False, stats=False,
                  launch: Optional[dict] = None, n_photons: Optional[int] = None, stream=None,
                  time_hist=None, time_bin_ns: float = 1.0, loss=False):
        """Queue one transport launch on the current (or given) stream.

        Returns a dict of device tensors: 'hit_map' int32 [events, channels]
        (accumulated into when passed in), and when requested 'grad' float64
        [events, channels, 4], 'records' uint8 [n, 96], 'stats' uint64 [24],
        'time_hist' int32 [events, bins] (time_hist = number of bins of width
        time_bin_ns, or a tensor to accumulate into) and 'loss' int64
        [n_groups + materials, 8] (loss = True or a tensor; needs
        set_loss_groups)."""
        ds = self.sources(src)
        n = ds.n_photons if n_photons is None else int(n_photons)
        dev = self.device
        if hit_map is None:
            hit_map = torch.zeros((ds.n_events, self.n_channels), dtype=torch.int32, device=dev)
        out = {"hit_map": hit_map}
        g = (torch.zeros((ds.n_events, self.n_channels, 4), dtype=torch.float64, device=dev)
             if grad is True else (grad if isinstance(grad, torch.Tensor) else None))
        if g is not None:
            out["grad"] = g
        rec = torch.empty((n, RECORD_DTYPE.itemsize), dtype=torch.uint8, device=dev) if records else None
        if rec is not None:
            out["records"] = rec
        st = torch.zeros(24, dtype=torch.int64, device=dev) if stats else None
        if st is not None:
            out["stats"] = st
        th = None
        if isinstance(time_hist, torch.Tensor):
            th = time_hist
        elif time_hist:
            th = torch.zeros((ds.n_events, int(time_hist)), dtype=torch.int32, device=dev)
        if th is not None:
            out["time_hist"] = th
        lt = None
        if isinstance(loss, torch.Tensor):
            lt = loss
        elif loss:
            lt = torch.zeros((getattr(self, "n_groups", 0) + len(self.materials), 8),
                             dtype=torch.int64, device=dev)
        if lt is not None:
            out["loss"] = lt
        extra = None
        if th is not None or lt is not None:
            extra = ExtraTallies(d_time_hist=_ptr(th), n_time_bins=th.shape[-1] if th is not None else 0,
                                 time_bin_ns=float(time_bin_ns), d_loss=_ptr(lt))
        lc = launch_cfg(launch)
        s = stream if stream is not None else current_stream(dev)
        sstruct = ds.struct(n)
        rp = self.run_params(seed, pid_base, max_steps, eps, grad_material)
        check(self.lib.xp_propagate_ex(self.ctx, ctypes.byref(sstruct), ctypes.byref(rp),
                                       _ptr(hit_map), _ptr(g), _ptr(rec), _ptr(st),
                                       ctypes.byref(extra) if extra else None,
                                       ctypes.byref(lc) if lc else None, ctypes.c_void_p(s)),
              self.ctx)
        out["_keep"] = ds
        return out

    def propagate_static(self, src, hit_map: torch.Tensor, seed=0, pid_base=0, max_steps=10_000,
                         eps=0.0, grad_material=0, grad: Optional[torch.Tensor] = None,
                         records: Optional[torch.Tensor] = None,
                         stats: Optional[torch.Tensor] = None, launch: Optional[dict] = None,
                         n_photons: Optional[int] = None, stream=None):
        """xp_propagate_static: the forward launch with its work counter and
        traversal-stack overflow area in the library's fixed device scratch.
        Every output is the caller's tensor (hit map int32 [events, channels],
        optional FP64 grad [events, channels, 4], uint8 records [n, 96], int64
        stats [24]) and src should already be device sources (self.sources),
        so that neither this call nor the library allocates."""
        ds = self.sources(src)
        n = ds.n_photons if n_photons is None else int(n_photons)
        lc = launch_cfg(launch)
        s = stream if stream is not None else current_stream(self.device)
        sstruct = ds.struct(n)
        rp = self.run_params(seed, pid_base, max_steps, eps, grad_material)
        check(self.lib.xp_propagate_static(self.ctx, ctypes.byref(sstruct), ctypes.byref(rp),
                                           _ptr(hit_map), _ptr(grad), _ptr(records), _ptr(stats),
                                           ctypes.byref(lc) if lc else None, ctypes.c_void_p(s)),
              self.ctx)

    def backward(self, src, grad_hits: torch.Tensor, seed=0, pid_base=0, max_steps=10_000,
                 eps=0.0, grad_material=0, grad_params: Optional[torch.Tensor] = None,
                 launch: Optional[dict] = None, stream=None) -> torch.Tensor:
        ds = self.sources(src)
        gh = grad_hits.to(device=self.device, dtype=torch.float32).contiguous()
        if gh.numel() != ds.n_events * self.n_channels:
            raise ValueError("grad_hits must have n_events * n_channels elements")
        gp = grad_params if grad_params is not None else torch.zeros(4, dtype=torch.float64,
                                                                     device=self.device)
        lc = launch_cfg(launch)
        s = stream if stream is not None else current_stream(self.device)
        sstruct = ds.struct()
        rp = self.run_params(seed, pid_base, max_steps, eps, grad_material)
        check(self.lib.xp_backward(self.ctx, ctypes.byref(sstruct), ctypes.byref(rp), _ptr(gh),
                                   _ptr(gp), ctypes.byref(lc) if lc else None, ctypes.c_void_p(s)),
              self.ctx)
        self._keep_bwd = (ds, gh)
        return gp

    def autotune(self, src, sample_photons=2_000_000, seed=0, grad_material=0, stream=None) -> dict:
        ds = self.sources(src)
        out = LaunchCfg()
        s = stream if stream is not None else current_stream(self.device)
        sstruct = ds.struct()
        rp = self.run_params(seed, 0, 10_000, 0.0, grad_material)
        check(self.lib.xp_autotune(self.ctx, ctypes.byref(sstruct), ctypes.byref(rp),
                                   int(sample_photons), ctypes.byref(out), ctypes.c_void_p(s)),
              self.ctx)
        return out.as_dict()

    def closest_hit(self, orig: torch.Tensor, dirs: torch.Tensor, tmin=0.0, tmax=math.inf,
                    skip: Optional[torch.Tensor] = None, brute=False, stream=None):
        o = orig.to(self.device, torch.float32).contiguous()
        d = dirs.to(self.device, torch.float32).contiguous()
        n = o.shape[0]
        sk = None if skip is None else skip.to(self.device, torch.int32).contiguous()
        tri = torch.empty(n, dtype=torch.int32, device=self.device)
        t = torch.empty(n, dtype=torch.float32, device=self.device)
        s = stream if stream is not None else current_stream(self.device)
        check(self.lib.xp_closest_hit(self.ctx, n, _ptr(o), _ptr(d), _ptr(sk), float(tmin),
                                      float(tmax), 1 if brute else 0, _ptr(tri), _ptr(t),
                                      ctypes.c_void_p(s)), self.ctx)
        return tri, t


def launch_cfg(launch: Optional[dict]):
    """The xp_launch_cfg of a launch-configuration dict, or None for the
    context's configuration.  Fields the dict leaves out take the library's
    defaults: 0 for every field but lds_levels, whose default is -1 (0 would
    stage no BVH levels in LDS)."""
    if not launch:
        return None
    return LaunchCfg(**{"lds_levels": -1, **launch})


def bvh_build_host(vertices, triangles, max_leaf_size=1, sah_bins=32, split_budget=0.0):
    """Build the BVH on the host only (xp_bvh_build_host; no device needed).
    Returns (info dict, nodes as NODE_DTYPE, records as TRIREC_DTYPE)."""
    lib = load()
    v = np.ascontiguousarray(vertices, dtype=np.float32).reshape(-1, 3)
    t = np.ascontiguousarray(triangles, dtype=np.int32).reshape(-1, 3)
    opts = BvhOptions(max_leaf_size, sah_bins, split_budget)
    info = BvhInfo()
    args = (_host_ptr(v), len(v), _host_ptr(t), len(t), ctypes.byref(opts), ctypes.byref(info))
    check(lib.xp_bvh_build_host(*args, None, 0, None, 0))
    nodes = np.zeros(info.n_nodes, dtype=_lib.NODE_DTYPE)
    recs = np.zeros(3 * info.n_references, dtype=_lib.TRIREC_DTYPE)
    check(lib.xp_bvh_build_host(*args, _host_ptr(nodes), len(nodes), _host_ptr(recs), len(recs)))
    d = {k: getattr(info, k) for k, _ in BvhInfo._fields_}
    return d, nodes, recs


def time_quantile(time_hist: torch.Tensor, time_bin_ns: float, q: float = 0.9, stream=None):
    """Per-event arrival-time quantile (q = 0.9: t90) of int32 time histograms
    [events, bins], computed on the device.  Returns float32 [events]."""
    lib = load()
    h = time_hist.contiguous()
    ne, nb = (1, h.shape[0]) if h.dim() == 1 else (h.shape[0], h.shape[1])
    out = torch.empty(ne, dtype=torch.float32, device=h.device)
    s = stream if stream is not None else current_stream(h.device)
    check(lib.xp_time_quantile(_ptr(h), int(ne), int(nb), float(time_bin_ns), float(q), _ptr(out),
                               ctypes.c_void_p(s)))
    return out


def sample_emission_time(seed, pid0, n, tau_singlet_ns, tau_triplet_ns, singlet_fraction,
                         device="cuda"):
    """Device emission-time sampler with the transport's schedule (test hook)."""
    lib = load()
    dev = torch.device(device)
    t = torch.empty(n, dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    check(lib.xp_sample_emission_time(int(seed), int(pid0), int(n), float(tau_singlet_ns),
                                      float(tau_triplet_ns), float(singlet_fraction), _ptr(t),
                                      _ptr(st), ctypes.c_void_p(current_stream(dev))))
    return t, st


def sample_wavelength(seed, pid0, n, mean_nm, fwhm_nm, device="cuda"):
    """Device emission-wavelength sampler with the transport's schedule (test hook)."""
    lib = load()
    dev = torch.device(device)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    check(lib.xp_sample_wavelength(int(seed), int(pid0), int(n), float(mean_nm), float(fwhm_nm),
                                   _ptr(out), ctypes.c_void_p(current_stream(dev))))
    return out


def surface_reflectance(model, n1, n_re, n_im, cos_i: torch.Tensor, film_n=0.0, film_d_nm=0.0,
                        lam=174.8):
    """|r_s|^2, |r_p|^2 of a complex-index / thin-film surface on the device (test hook)."""
    lib = load()
    c = cos_i.to(torch.float32).contiguous()
    rs, rp = torch.empty_like(c), torch.empty_like(c)
    check(lib.xp_surface_reflectance(int(model), float(n1), float(n_re), float(n_im), float(film_n),
                                     float(film_d_nm), float(lam), c.numel(), _ptr(c), _ptr(rs),
                                     _ptr(rp), ctypes.c_void_p(current_stream(c.device))))
    return rs, rp


def records_to_numpy(rec: torch.Tensor) -> np.ndarray:
    return rec.cpu().numpy().view(RECORD_DTYPE).reshape(-1)


def sample(kind, seed, pid0, n, in_dir=None, in_pol=None, cyl=(0.0, 0.0, 0.0), device="cuda"):
    """Device samplers with the transport's random-number schedule (test hook)."""
    lib = load()
    dev = torch.device(device)

    def rows(x):
        if x is None:
            return None
        t = torch.as_tensor(np.asarray(x, dtype=np.float32), device=dev)
        return t.expand(n, 3).contiguous() if t.dim() == 1 else t.contiguous()

    di, pi = rows(in_dir), rows(in_pol)
    od = torch.empty((n, 3), dtype=torch.float32, device=dev)
    op = torch.empty((n, 3), dtype=torch.float32, device=dev)
    check(lib.xp_sample(int(kind), int(seed), int(pid0), int(n), _ptr(di), _ptr(pi),
                        float(cyl[0]), float(cyl[1]), float(cyl[2]), _ptr(od), _ptr(op),
                        ctypes.c_void_p(current_stream(dev))))
    return od, op
