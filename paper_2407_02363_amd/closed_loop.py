"""Closed-loop collision avoidance (Alg. 2 feeding Sec. III-F), through the
C-ABI: every control step inserts the current obstacle cloud into the map,
computes the exact EDT, queries the arm's bounding spheres, and hands the
closest obstacle points to the task-priority controller, whose joint
velocity moves the arm for one control period.  Only orchestration lives
here: the map steps run in the library's kernels, the control step in its
host code, the forward kinematics in the arm model."""
from __future__ import annotations

import time

import numpy as np
import torch

from . import controller, edt, inputs

# The arm's workspace: 2.56 m on a side at 1 cm.  The arm stands at the middle
# of the floor plane and reaches under 2 m up, so every bounding sphere stays
# inside the map (a sphere outside it only gets a conservative zero distance).
ARM_GRID = inputs.Grid(256, 256, 256, (0.0, 0.0, 0.0), 0.01)


def ball_points(centre, radius, n=4000, seed=0, step=0.005):
    """Points of a solid ball (map frame): n points on its surface plus a
    lattice of spacing `step` inside it."""
    g = inputs.rng(seed)
    v = g.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    k = int(radius / step)
    ax = np.arange(-k, k + 1) * step
    lat = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    lat = lat[np.linalg.norm(lat, axis=1) < radius]
    return (np.asarray(centre) + np.vstack([radius * v, lat])).astype(np.float32)


class ClosedLoop:
    def __init__(self, ci, grid=ARM_GRID, device="cuda:0", margin=0.05, buffer=0.02, target_offset=0.05, gain=10.0,
                 hold_gain=2.0, qdot_max=2.0, dt=0.002):
        self.ci = ci
        self.g = grid
        self.dev = torch.device(device)
        d = self.dev
        n = self.g.n
        self.occ = torch.zeros(n, dtype=torch.uint8, device=d)
        self.d2 = torch.empty(n, dtype=torch.int32, device=d)
        self.site = torch.empty(n, dtype=torch.int32, device=d)
        m = len(ci.sphere_radii)
        self.radii = torch.from_numpy(np.asarray(ci.sphere_radii, np.float32)).to(d)
        self.centres = torch.zeros((m, 3), dtype=torch.float32, device=d)
        self.out = edt.new_query_out(m, d)
        self.host = torch.empty(self.out.shape, dtype=torch.int32, pin_memory=True)
        self.eye = torch.tensor([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], dtype=torch.float32, device=d)
        self.x_m = np.asarray(ci.sphere_radii, np.float64) + margin
        self.count = np.asarray(ci.sphere_links, np.int32)   # a sphere on link L moves with joints 1..L
        self.params = dict(buffer=buffer, target_offset=target_offset, gain=gain)
        self.hold_gain, self.qdot_max, self.dt = hold_gain, qdot_max, dt

    def run(self, q0, obstacle, steps, avoid=True):
        """obstacle(t) -> float32 [k, 3] map-frame points.  Returns per-step
        minimum clearance (x_i - r_i over the spheres, metres), the joint
        trajectory and the mean wall time per step."""
        robot = self.ci.robot
        q = np.array(q0, np.float64)
        clear, traj = [], []
        t0 = time.perf_counter()
        for k in range(steps):
            t = k * self.dt
            C = inputs.sphere_centres(robot, q, self.ci.sphere_links, self.ci.sphere_local)
            self.centres.copy_(torch.from_numpy(np.asarray(C, np.float32)))
            pts = torch.from_numpy(obstacle(t)).to(self.dev)
            edt.edt_clear(self.g, self.occ)
            edt.edt_insert_points(self.g, self.occ, pts, self.eye)
            edt.edt_compute(self.g, self.occ, self.d2, self.site)
            edt.edt_query_spheres(self.g, self.d2, self.site, self.centres, self.radii, self.out)
            self.host.copy_(self.out)          # synchronous: the controller needs it now
            rec = self.host.numpy()
            flags = rec[:, 5]
            O = rec[:, 12:15].view(np.float32).astype(np.float64)
            far = (flags & (edt.Q_EMPTY | edt.Q_OUT_OF_MAP)) != 0
            O[far] = np.asarray(C, np.float64)[far] + 10.0     # nothing near: an inactive task
            qdot0 = self.hold_gain * (np.asarray(q0) - q)
            if avoid:
                axes, origins = robot.joint_frames(q)
                qdot, _, x = controller.tp_step(axes, origins, self.count, C, O, self.x_m, qdot0=qdot0,
                                                **self.params)
            else:
                qdot = qdot0
                x = np.linalg.norm(O - np.asarray(C, np.float64), axis=1)
            clear.append(float((x - np.asarray(self.ci.sphere_radii, np.float64)).min()))
            qdot = np.clip(qdot, -self.qdot_max, self.qdot_max)
            q = q + qdot * self.dt
            traj.append(q.copy())
        return np.array(clear), np.array(traj), (time.perf_counter() - t0) / steps


def fly_through(ci, q0, link=4, speed=0.5, radius=0.06, duration=1.5, miss=0.05, seed=0):
    """A ball of the given radius flying at `speed` along the map's x axis,
    its centre passing `miss` metres (along y) from the centre of a sphere
    on `link` of the arm at state q0, at half time: with the arm held still
    the ball cuts through it."""
    robot = ci.robot
    C = inputs.sphere_centres(robot, q0, ci.sphere_links, ci.sphere_local)
    i = int(np.flatnonzero(np.asarray(ci.sphere_links) == link)[0])
    target = np.asarray(C[i], np.float64)
    start = target - np.array([speed * duration / 2, 0.0, 0.0]) + np.array([0.0, miss, 0.0])
    shape = ball_points((0.0, 0.0, 0.0), radius, seed=seed)

    def obstacle(t):
        return (shape + (start + np.array([speed * t, 0.0, 0.0]))).astype(np.float32)

    return obstacle
