"""One control cycle of Alg. 2 on the GPU, driven through the C-ABI binding.

Per cycle: ClearMap of the self map M_S and the environment map M_I; insert
the robot links placed by the cycle's joint state into M_S; insert the
cycle's point cloud into M_I, skipping voxels M_S occupies (Sec. III-A);
compute the exact EDT of both maps; extract the closest obstacle at each
sphere centre in both maps.  Only orchestration lives here: every step is
a library call, and all inputs are staged in device memory beforehand.
"""
from __future__ import annotations

import numpy as np
import torch

from . import edt


class ControlCycle:
    EDT_MODES = ("many", "per_map", "batched")

    def __init__(self, ci, device="cuda:0", self_mask: int = 0xFF, centres=None,
                 edt_mode: str = "many", two_streams: bool = False):
        """ci: inputs.CycleInputs.  centres: float32 [S, m, 3] per joint
        state (computed from ci.joint_states by forward kinematics if None).
        edt_mode: how the two maps' EDTs run (same results every way):
          "many"     one edt_compute_many for both maps (one launch per pass,
                     the second map's tiles fill the first one's tail);
          "per_map"  one edt_compute per map;
          "batched"  one persistent edt_compute_batched launch.
        two_streams ("per_map" only): run the environment map's steps on a
        second stream forked from and joined back into the caller's stream;
        the point insertion still waits for the self map it excludes."""
        from . import inputs
        self.ci = ci
        self.grid = ci.grid
        self.dev = torch.device(device)
        self.self_mask = int(self_mask)
        n = ci.grid.n
        d = self.dev
        # both occupancy maps in one buffer, so that one clear over a grid of
        # twice the depth zeroes both
        self.occ_both = torch.zeros(2 * n, dtype=torch.uint8, device=d)
        self.occ_env = self.occ_both[:n]
        self.occ_self = self.occ_both[n:]
        g = ci.grid
        self.grid2 = inputs.Grid(g.nx, g.ny, 2 * g.nz, g.origin, g.voxel)
        self.d2_self = torch.empty(n, dtype=torch.int32, device=d)
        self.site_self = torch.empty(n, dtype=torch.int32, device=d)
        self.d2_env = torch.empty(n, dtype=torch.int32, device=d)
        self.site_env = torch.empty(n, dtype=torch.int32, device=d)
        self.frames = torch.from_numpy(np.stack(ci.frames)).to(d)           # [F, n, 3]
        self.T = torch.from_numpy(ci.T_map_cam).to(d)
        self.link_pts = torch.from_numpy(ci.link_pts).to(d)
        self.link_off = np.asarray(ci.link_off, np.int32)
        states = ci.joint_states
        self.poses = torch.from_numpy(np.stack([ci.robot.poses12(q) for q in states])).to(d)
        if centres is None:
            centres = np.stack([inputs.sphere_centres(ci.robot, q, ci.sphere_links, ci.sphere_local)
                                for q in states])
        self.centres_host = centres
        self.centres = torch.from_numpy(np.ascontiguousarray(centres, np.float32)).to(d)
        self.radii = torch.from_numpy(np.asarray(ci.sphere_radii, np.float32)).to(d)
        m = self.radii.numel()
        self.out_env = edt.new_query_out(m, d)
        self.out_self = edt.new_query_out(m, d)
        self.n_frames = self.frames.shape[0]
        self.n_states = self.poses.shape[0]
        if edt_mode not in self.EDT_MODES:
            raise ValueError(f"edt_mode must be one of {self.EDT_MODES}")
        self.edt_mode = edt_mode
        self.two_streams = bool(two_streams) and edt_mode == "per_map"
        if self.two_streams:
            self.side = torch.cuda.Stream(device=d)
            self.ev_fork = torch.cuda.Event()
            self.ev_links = torch.cuda.Event()
            self.ev_join = torch.cuda.Event()
        self.maps = edt.batch_maps([ci.grid, ci.grid], [self.occ_env, self.occ_self],
                                   [self.d2_env, self.d2_self], [self.site_env, self.site_self])
        if edt_mode == "batched":
            self.batch_ws = edt.new_batch_workspace(2, d)

    @property
    def voxels_per_cycle(self) -> int:
        return 2 * self.grid.n

    def run(self, k: int, stream=None):
        """Enqueue cycle k (frame k mod F, joint state k mod S)."""
        if self.two_streams:
            return self._run_two_streams(k, stream)
        g = self.grid
        f = k % self.n_frames
        s = k % self.n_states
        joint = self.edt_mode != "per_map"   # one clear and one query launch for both maps
        if joint:
            edt.edt_clear(self.grid2, self.occ_both, stream)
        else:
            edt.edt_clear(g, self.occ_self, stream)
            edt.edt_clear(g, self.occ_env, stream)
        edt.edt_insert_links(g, self.occ_self, self.link_pts, self.link_off, self.poses[s],
                             self.self_mask, stream)
        edt.edt_insert_points(g, self.occ_env, self.frames[f], self.T, exclude=self.occ_self,
                              stream=stream)
        if self.edt_mode == "many":
            edt.edt_compute_many(self.maps, stream=stream)
        elif self.edt_mode == "batched":
            edt.edt_compute_batched(self.maps, self.batch_ws, stream=stream)
        else:
            edt.edt_compute(g, self.occ_env, self.d2_env, self.site_env, stream=stream)
            edt.edt_compute(g, self.occ_self, self.d2_self, self.site_self, stream=stream)
        if joint:
            c = self.centres[s]
            edt.edt_query_spheres_many(self.maps, [c, c], [self.radii, self.radii],
                                       [self.out_env, self.out_self], stream)
        else:
            edt.edt_query_spheres(g, self.d2_env, self.site_env, self.centres[s], self.radii,
                                  self.out_env, stream)
            edt.edt_query_spheres(g, self.d2_self, self.site_self, self.centres[s], self.radii,
                                  self.out_self, stream)

    def _run_two_streams(self, k: int, stream=None):
        g = self.grid
        f = k % self.n_frames
        s = k % self.n_states
        main = stream if stream is not None else torch.cuda.current_stream(self.dev)
        side = self.side
        self.ev_fork.record(main)
        side.wait_event(self.ev_fork)
        # self map on the caller's stream
        edt.edt_clear(g, self.occ_self, main)
        edt.edt_insert_links(g, self.occ_self, self.link_pts, self.link_off, self.poses[s],
                             self.self_mask, main)
        self.ev_links.record(main)
        # environment map on the side stream, its insertion after the links
        edt.edt_clear(g, self.occ_env, side)
        side.wait_event(self.ev_links)
        edt.edt_insert_points(g, self.occ_env, self.frames[f], self.T, exclude=self.occ_self,
                              stream=side)
        edt.edt_compute(g, self.occ_env, self.d2_env, self.site_env, stream=side)
        edt.edt_query_spheres(g, self.d2_env, self.site_env, self.centres[s], self.radii,
                              self.out_env, side)
        edt.edt_compute(g, self.occ_self, self.d2_self, self.site_self, stream=main)
        edt.edt_query_spheres(g, self.d2_self, self.site_self, self.centres[s], self.radii,
                              self.out_self, main)
        self.ev_join.record(side)
        main.wait_event(self.ev_join)

    # -- the two-stream cycle replayed from three single-stream graphs per
    # slot: [clear + insert the self map] on the caller's stream, then
    # [clear, insert, EDT, query of the environment map] on the side stream
    # once the self map is in, and [EDT, query of the self map] on the
    # caller's stream, which finally waits for the side stream.
    def _self_links(self, s, stream=None):
        edt.edt_clear(self.grid, self.occ_self, stream)
        edt.edt_insert_links(self.grid, self.occ_self, self.link_pts, self.link_off, self.poses[s],
                             self.self_mask, stream)

    def _env_all(self, f, s, stream=None):
        g = self.grid
        edt.edt_clear(g, self.occ_env, stream)
        edt.edt_insert_points(g, self.occ_env, self.frames[f], self.T, exclude=self.occ_self,
                              stream=stream)
        edt.edt_compute(g, self.occ_env, self.d2_env, self.site_env, stream=stream)
        edt.edt_query_spheres(g, self.d2_env, self.site_env, self.centres[s], self.radii,
                              self.out_env, stream)

    def _self_edt(self, s, stream=None):
        g = self.grid
        edt.edt_compute(g, self.occ_self, self.d2_self, self.site_self, stream=stream)
        edt.edt_query_spheres(g, self.d2_self, self.site_self, self.centres[s], self.radii,
                              self.out_self, stream)

    def capture_split_graphs(self, n_graphs: int):
        """Three graphs per slot k < n_graphs (see replay_split)."""
        if not hasattr(self, "side"):
            self.side = torch.cuda.Stream(device=self.dev)
            self.ev_links = torch.cuda.Event()
            self.ev_join = torch.cuda.Event()
        torch.cuda.synchronize(self.dev)
        parts = []
        for k in range(n_graphs):
            f, s = k % self.n_frames, k % self.n_states
            trio = []
            for fn in (lambda: self._self_links(s), lambda: self._env_all(f, s),
                       lambda: self._self_edt(s)):
                fn()
                torch.cuda.synchronize(self.dev)
                gr = torch.cuda.CUDAGraph()
                with torch.cuda.graph(gr, capture_error_mode="thread_local"):
                    fn()
                trio.append(gr)
            parts.append(tuple(trio))
        torch.cuda.synchronize(self.dev)
        self.split_graphs = parts
        return parts

    def replay_split(self, k: int):
        """Cycle k from the split graphs, on the current stream plus the side
        stream (joined back before returning)."""
        g_links, g_env, g_self = self.split_graphs[k % len(self.split_graphs)]
        main = torch.cuda.current_stream(self.dev)
        g_links.replay()
        self.ev_links.record(main)
        self.side.wait_event(self.ev_links)
        with torch.cuda.stream(self.side):
            g_env.replay()
        self.ev_join.record(self.side)
        g_self.replay()
        main.wait_event(self.ev_join)

    def capture_graphs(self, n_graphs: int):
        """One HIP graph per (frame, state) slot k < n_graphs, each replaying
        the whole cycle k; warm-up runs first so nothing initialises inside
        the capture."""
        torch.cuda.synchronize(self.dev)
        for k in range(min(n_graphs, 3)):
            self.run(k)
        torch.cuda.synchronize(self.dev)
        graphs = []
        for k in range(n_graphs):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, capture_error_mode="thread_local"):
                self.run(k)
            graphs.append(g)
        torch.cuda.synchronize(self.dev)
        return graphs
