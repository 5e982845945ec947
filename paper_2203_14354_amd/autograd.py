"""Score-function gradients of the expected hit map behind torch.autograd.

The parameters are the four optical quantities of the paper's systematic
study (table tab:lce_sys): the absorption length and the Rayleigh length of
one material, the total reflectivity of the surfaces tagged "reflectivity"
(its diffuse/specular split kept), and the transparency of the surfaces tagged
"transparency".  The expected hits E[H] are estimated by the transported
photon counts; their Jacobian by the path-reweighting (likelihood-ratio)
scores tallied per detected photon in FP64:

  d log p / d L_abs = L / L_abs^2
  d log p / d L_R   = L / L_R^2 - N_scatter / L_R
  d log p / d R     = (reflections on tagged surfaces) / R
  d log p / d T     = (transmissions through tagged surfaces) / T

Two backward modes: 'fused' keeps the Jacobian tallied by the forward launch
and contracts it with the upstream gradient; 'replay' re-runs the same photon
histories (same seed and photon ids) in the backward kernel, which needs no
Jacobian storage (for hit maps with many cells).
"""
from __future__ import annotations

import copy
from typing import Optional

import torch

from . import workloads as W


def apply_params(det, params, grad_material=0):
    """Set the detector's tables to the parameter values (L_abs, L_R, R, T)."""
    p = [float(x) for x in params]
    mats = copy.deepcopy(det.mesh.materials)
    if grad_material >= 0:
        mats[grad_material] = W.Material(mats[grad_material].n, p[0], p[1])
    surfs = copy.deepcopy(det.mesh.surfaces)
    for s in surfs:
        if s.grad_param == W.GRAD_REFLECTIVITY:
            r_old = s.r_diffuse + s.r_specular
            frac = s.r_specular / r_old if r_old > 0 else 0.0
            s.r_specular = p[2] * frac
            s.r_diffuse = p[2] - s.r_specular
            s.p_absorb = 1.0 - s.p_detect - s.p_transmit - p[2]
        elif s.grad_param == W.GRAD_TRANSPARENCY:
            s.p_absorb = 1.0 - s.p_detect - s.r_diffuse - s.r_specular - p[3]
            s.p_transmit = p[3]
    det.set_materials(mats)
    det.set_surfaces(surfs)


class XeHits(torch.autograd.Function):
    """hits = XeHits.apply(params, det, sources, seed, mode) -> float64 [events, channels].

    params: float64 tensor (L_abs, L_R, R, T); det: runtime.Detector; sources:
    workloads.Sources or runtime.DeviceSources; mode: 'fused' or 'replay'."""

    @staticmethod
    def forward(ctx, params, det, sources, seed=0, mode="fused", grad_material=0):
        apply_params(det, params.detach().cpu(), grad_material)
        ds = det.sources(sources)
        fused = mode == "fused"
        out = det.propagate(ds, seed=seed, grad=fused, grad_material=grad_material)
        ctx.det, ctx.ds, ctx.seed, ctx.mode, ctx.gm = det, ds, seed, mode, grad_material
        ctx.params = params.detach().cpu().clone()
        ctx.params_device = params.device
        if fused:
            ctx.save_for_backward(out["grad"])
        return out["hit_map"].to(torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        if ctx.mode == "fused":
            (G,) = ctx.saved_tensors
            gp = torch.einsum("ec,ecp->p", grad_out.to(torch.float64), G)
        else:
            apply_params(ctx.det, ctx.params, ctx.gm)
            gp = ctx.det.backward(ctx.ds, grad_out, seed=ctx.seed, grad_material=ctx.gm)
        return gp.to(ctx.params_device), None, None, None, None, None


def hits(params: torch.Tensor, det, sources, seed=0, mode="fused", grad_material=0):
    return XeHits.apply(params, det, sources, seed, mode, grad_material)


def base_params(mesh, grad_material=0) -> torch.Tensor:
    """(L_abs, L_R, R, T) as currently set in the mesh's tables."""
    m = mesh.materials[grad_material]
    R = next((s.r_diffuse + s.r_specular for s in mesh.surfaces
              if s.grad_param == W.GRAD_REFLECTIVITY), 1.0)
    T = next((s.p_transmit for s in mesh.surfaces if s.grad_param == W.GRAD_TRANSPARENCY), 1.0)
    return torch.tensor([m.abs_length, m.rayleigh_length, R, T], dtype=torch.float64)
