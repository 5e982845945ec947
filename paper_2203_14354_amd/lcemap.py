"""Light-collection-efficiency map with gradients.

The paper maps the LCE over the TPC with point sources on a grid (section
"Light collection efficiency", about 2,500 positions of 1e6 photons each).
Here every cell of an equal-volume (R^2, phi, z) grid is one source and one
event; a sensor -> {top, bottom} channel map folds the hit map to two columns,
and the FP64 gradient tallies give, per cell and array, the derivative of the
expected counts with respect to (L_abs, L_R, R, T).  Cells are processed in
batches of launches; photon ids are global (cell * photons_per_cell + k), so
the result does not depend on the batch size.
"""
from __future__ import annotations

import numpy as np
import torch

from . import workloads as W


def lce_map(det, centroids: np.ndarray, photons_per_cell: int, seed: int = 0,
            batch_cells: int = 16384, grad: bool = True, grad_material: int = 0, launch=None):
    """Returns (hits int32 [cells, channels], grad float64 [cells, channels, 4] or None)."""
    cells = int(len(centroids))
    dev = det.device
    hits = torch.zeros((cells, det.n_channels), dtype=torch.int32, device=dev)
    g = torch.zeros((cells, det.n_channels, 4), dtype=torch.float64, device=dev) if grad else None
    for c0 in range(0, cells, batch_cells):
        c1 = min(cells, c0 + batch_cells)
        src = W.point_sources(centroids[c0:c1], count_per_source=photons_per_cell,
                              per_source_events=True)
        det.propagate(src, seed=seed, pid_base=c0 * photons_per_cell, hit_map=hits[c0:c1],
                      grad=g[c0:c1] if grad else False, grad_material=grad_material,
                      launch=launch)
    return hits, g


def tpc1_lce_map_detector(device=0, plane=True):
    """The small TPC (with the transparent plane) with its 38 sensors folded
    into the two arrays (channel 0 top, 1 bottom)."""
    from .runtime import Detector
    mesh = W.tpc1(plane=plane)
    return Detector(mesh, device=device, channel_of_sensor=W.tpc1_top_bottom_channels(mesh),
                    n_channels=2)
