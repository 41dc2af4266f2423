"""Exact self-map distances at the arm's sphere centres for many joint states.

For each state (Alg. 2 steps for the self map): ClearMap, insert the voxel
models of the obstacle links O_L placed by the state's forward kinematics,
compute the exact EDT, and read sqrt(d2) at every sphere centre
(ExtractClosestObstaclePose).  States go in chunks of up to EDT_BATCH_MAX
maps, each step one launch (or one per pass) for the whole chunk:
edt_clear_insert_links_many, edt_compute_many (edt_mode="batched" uses the
persistent batched launch), edt_query_spheres_many; and the whole chunk is
replayed from a HIP graph whose pose and centre buffers are refilled before
every replay.  Graphs exist for chunk sizes 1, 2, 4, ... and the full
chunk, so a partial chunk (the states the surrogate could not clear, for
instance) costs the next size up rather than a full chunk.  These distances are the
surrogate's labels and the measure of its error; the same path is the
fallback when the surrogate is not trusted.
Only orchestration lives here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import edt, inputs


class SelfMapLabeler:
    def __init__(self, setup: "inputs.SelfMapSetup", chunk: int = 48, device="cuda:0",
                 use_graph: bool = True, edt_mode: str = "many"):
        if edt_mode not in ("many", "batched"):
            raise ValueError("edt_mode must be 'many' or 'batched'")
        self.edt_mode = edt_mode
        self.s = setup
        self.chunk = int(chunk)
        self.dev = torch.device(device)
        d = self.dev
        g = setup.grid
        n = g.n
        c = self.chunk
        self.occ = [torch.zeros(n, dtype=torch.uint8, device=d) for _ in range(c)]
        self.d2 = [torch.empty(n, dtype=torch.int32, device=d) for _ in range(c)]
        self.site = [torch.empty(n, dtype=torch.int32, device=d) for _ in range(c)]
        self.poses = torch.zeros((c, setup.robot.n_links, 12), dtype=torch.float32, device=d)
        self.centres = torch.zeros((c, len(setup.sphere_radii), 3), dtype=torch.float32, device=d)
        self.radii = torch.from_numpy(setup.sphere_radii).to(d)
        self.out = torch.empty((c, len(setup.sphere_radii), edt.SPHERE_RESULT_WORDS),
                               dtype=torch.int32, device=d)
        self.link_pts = torch.from_numpy(setup.link_pts).to(d)
        # per-slot switches of the gated transform (run_chunk(gated=True)):
        # slot i is transformed only while gate[i] != 0, a value kernels
        # earlier in the stream may write
        self.gate = torch.ones(c, dtype=torch.int32, device=d)
        sizes = [1 << k for k in range(7) if (1 << k) < c] + [c]
        self.maps = {k: edt.batch_maps([g] * k, self.occ[:k], self.d2[:k], self.site[:k])
                     for k in sizes}
        self.ws = edt.new_batch_workspace(c, d)
        self.graphs = {}
        if use_graph:
            for k in sizes:
                self.run_chunk(k)
            torch.cuda.synchronize(d)
            for k in sizes:
                gr = torch.cuda.CUDAGraph()
                with torch.cuda.graph(gr, capture_error_mode="thread_local"):
                    self.run_chunk(k)
                self.graphs[k] = gr
            torch.cuda.synchronize(d)

    def size_for(self, k: int) -> int:
        """Smallest chunk size with a batch plan that holds k states."""
        return min(s for s in self.maps if s >= k)

    def run_chunk(self, k=None, stream=None, gated=False):
        """Clear, insert, transform and query the first k maps (k must be a
        planned size; None = the full chunk).  gated: the transform skips
        every slot whose gate is 0 (its distances are then stale)."""
        g = self.s.grid
        k = self.chunk if k is None else k
        gates = self.gate[:k] if gated else None
        edt.edt_clear_insert_links_many(g, self.occ[:k], self.link_pts, self.s.link_off, self.poses[:k],
                                        self.s.mask, gates, stream)
        if gated:
            edt.edt_compute_many_gated(self.maps[k], self.gate[:k], stream=stream)
        elif self.edt_mode == "many":
            edt.edt_compute_many(self.maps[k], stream=stream)
        else:
            edt.edt_compute_batched(self.maps[k], self.ws, stream=stream)
        edt.edt_query_spheres_many(self.maps[k], [self.centres[j] for j in range(k)], [self.radii] * k,
                                   [self.out[j] for j in range(k)], stream)

    def exact_view(self, k):
        """dist_vox of the last run's first k slots: float32 [k, m] view of
        the query records (strided, on the device)."""
        return self.out[:k, :, 6].view(torch.float32)

    def stage(self, qs: np.ndarray):
        """Host forward kinematics of many states -> device (poses, centres)."""
        f = self.s.robot.fk_batch(qs)
        poses = torch.from_numpy(f.reshape(len(qs), self.s.robot.n_links, 12).astype(np.float32))
        cen = inputs.sphere_centres_batch(self.s.robot, qs, self.s.sphere_links, self.s.sphere_local)
        return poses.to(self.dev), torch.from_numpy(cen).to(self.dev)

    def distances(self, poses_dev, centres_dev, out_dev=None):
        """sqrt(d2) (voxels) at every sphere centre for staged states:
        float32 [N, m] on the device."""
        n = poses_dev.shape[0]
        m = centres_dev.shape[1]
        res = out_dev if out_dev is not None else torch.empty((n, m), dtype=torch.float32,
                                                              device=self.dev)
        for s0 in range(0, n, self.chunk):
            k = min(self.chunk, n - s0)
            size = self.size_for(k)
            self.poses[:k].copy_(poses_dev[s0:s0 + k])
            self.centres[:k].copy_(centres_dev[s0:s0 + k])
            if k < size:   # the unused slots of the plan repeat the last state
                self.poses[k:size].copy_(poses_dev[s0 + k - 1].expand(size - k, -1, -1))
                self.centres[k:size].copy_(centres_dev[s0 + k - 1].expand(size - k, -1, -1))
            if size in self.graphs:
                self.graphs[size].replay()
            else:
                self.run_chunk(size)
            res[s0:s0 + k].copy_(self.out[:k, :, 6].view(torch.float32))
        return res

    def labels(self, qs: np.ndarray) -> torch.Tensor:
        poses, cen = self.stage(qs)
        return self.distances(poses, cen)
