"""Batched control cycle over many maps of uneven size, through the C-ABI.

Per cycle and map: ClearMap, insert that map's point cloud, the exact EDT,
and the sphere query at every look-ahead joint state's sphere centres; the
clear and insertion of every map is one pair of launches and the queries of
every map one launch (batched_io, the default), or one launch per map and
step.  Three ways to run the EDT of the batch:

  run_plain    one edt_compute per map (two kernels per map), and the clear,
               insertion and queries one launch per map as well
  run_batched  one edt_compute_batched for all maps (one persistent launch)
  run_many     one edt_compute_many for all maps (one launch per pass)

Either can be captured into a HIP graph.  Only orchestration lives here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import edt


class BatchCycle:
    def __init__(self, bi, device="cuda:0", batched_io: bool = True):
        """bi: inputs.BatchInputs.  batched_io: clear, insert and query every
        map in one launch each (edt_clear_insert_points_many,
        edt_query_spheres_many); False: one launch per map and step."""
        self.bi = bi
        self.batched_io = batched_io
        self.dev = torch.device(device)
        d = self.dev
        self.grids = list(bi.grids)
        self.n_maps = len(self.grids)
        self.occ = [torch.zeros(g.n, dtype=torch.uint8, device=d) for g in self.grids]
        self.d2 = [torch.empty(g.n, dtype=torch.int32, device=d) for g in self.grids]
        self.site = [torch.empty(g.n, dtype=torch.int32, device=d) for g in self.grids]
        self.clouds = [torch.from_numpy(np.ascontiguousarray(c)).to(d) for c in bi.clouds]
        self.T = [torch.from_numpy(np.asarray(t, np.float32)).to(d) for t in bi.T_map_cam]
        self.centres = [torch.from_numpy(np.ascontiguousarray(c.reshape(-1, 3), np.float32)).to(d)
                        for c in bi.centres]
        self.radii = [torch.from_numpy(np.tile(r, c.shape[0]).astype(np.float32)).to(d)
                      for r, c in zip(bi.sphere_radii, bi.centres)]
        self.out = [edt.new_query_out(r.numel(), d) for r in self.radii]
        self.maps = edt.batch_maps(self.grids, self.occ, self.d2, self.site)
        self.ws = edt.new_batch_workspace(self.n_maps, d)

    @property
    def voxels(self) -> int:
        return sum(g.n for g in self.grids)

    @property
    def queries(self) -> int:
        return sum(r.numel() for r in self.radii)

    def _insert(self, stream=None, batched=None):
        if self.batched_io if batched is None else batched:
            edt.edt_clear_insert_points_many(self.grids, self.occ, self.clouds, self.T, stream)
            return
        for g, o, c, t in zip(self.grids, self.occ, self.clouds, self.T):
            edt.edt_clear(g, o, stream)
            edt.edt_insert_points(g, o, c, t, stream=stream)

    def _query(self, stream=None, batched=None):
        if self.batched_io if batched is None else batched:
            edt.edt_query_spheres_many(self.maps, self.centres, self.radii, self.out, stream)
            return
        for i, g in enumerate(self.grids):
            edt.edt_query_spheres(g, self.d2[i], self.site[i], self.centres[i], self.radii[i],
                                  self.out[i], stream)

    def run_plain(self, stream=None):
        """The per-map loop: every step one launch per map."""
        self._insert(stream, batched=False)
        for g, o, d2, s in zip(self.grids, self.occ, self.d2, self.site):
            edt.edt_compute(g, o, d2, s, stream=stream)
        self._query(stream, batched=False)

    def run_batched(self, stream=None):
        self._insert(stream)
        edt.edt_compute_batched(self.maps, self.ws, stream=stream)
        self._query(stream)

    def run_many(self, stream=None):
        self._insert(stream)
        edt.edt_compute_many(self.maps, stream=stream)
        self._query(stream)

    def capture(self, fn):
        """HIP graph of one cycle (fn = run_plain, run_batched or run_many)."""
        fn()
        torch.cuda.synchronize(self.dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, capture_error_mode="thread_local"):
            fn()
        torch.cuda.synchronize(self.dev)
        return g
