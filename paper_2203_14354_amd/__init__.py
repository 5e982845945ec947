"""MI355X (gfx950) optical-photon transport for liquid-xenon TPCs.

Submodules:
  workloads  seeded synthetic detectors, optical tables and sources (inputs only)
  runtime    Detector / propagate / backward / autotune over the C ABI
  autograd   score-function gradients behind torch.autograd.Function
  batched    many uneven sources in one persistent launch under a HIP graph

The HIP library is loaded lazily by ``runtime``; importing this package does
not touch the GPU.
"""
__all__ = ["workloads", "runtime"]
