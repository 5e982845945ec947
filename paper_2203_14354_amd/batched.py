"""Many uneven sources in one persistent launch, replayed from a HIP graph.

The analogue of the paper's thousands of independent point-source runs
(section "Light collection efficiency": about 2,500 positions): every source
becomes one event (one hit-map row); the launch's photon ids are split among
sources by prefix sums of their photon counts, and the persistent kernel
balances the uneven counts across the whole GPU.  The launch configuration
is autotuned once; the launch (hit-map clear + work-counter reset + kernel)
is captured in a HIP graph through torch.cuda.graph and replayed.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch


class BatchedRunner:
    def __init__(self, det, sources, seed=0, pid_base=0, autotune=True, use_graph=True,
                 tune_photons=4_000_000):
        self.det = det
        self.ds = det.sources(sources)
        self.seed = seed
        self.pid_base = pid_base
        dev = det.device
        self.hit_map = torch.zeros((self.ds.n_events, det.n_channels), dtype=torch.int32,
                                   device=dev)
        self.launch = det.autotune(self.ds, sample_photons=tune_photons, seed=seed) if autotune \
            else None
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        if use_graph:
            # warm the allocator and the kernels on a side stream, then capture
            s = torch.cuda.Stream(device=dev)
            s.wait_stream(torch.cuda.current_stream(dev))
            with torch.cuda.stream(s):
                self._eager()
            torch.cuda.current_stream(dev).wait_stream(s)
            torch.cuda.synchronize(dev)
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self._eager()
            torch.cuda.synchronize(dev)

    def _eager(self):
        self.hit_map.zero_()  # a fill kernel, not a memset node
        self.det.propagate(self.ds, seed=self.seed, pid_base=self.pid_base,
                           hit_map=self.hit_map, launch=self.launch)

    def run(self) -> torch.Tensor:
        """One batched launch (graph replay when captured); returns the hit map."""
        if self.graph is not None:
            self.graph.replay()
        else:
            self._eager()
        return self.hit_map
