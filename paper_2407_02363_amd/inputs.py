"""Seeded synthetic inputs for the distance-map hot path.

This module produces inputs only: occupancy grids, depth-camera point
clouds, robot link voxel models, link poses and bounding-sphere centres.  It
holds none of the arithmetic the hot path computes (point insertion, the
distance transform, sphere queries), so both the HIP path and the CPU oracle
can consume it without sharing any of that arithmetic.  Everything is numpy,
seeded with PCG64, deterministic across machines.

The paper evaluates on live camera data of a lab scene (Sec. IV-A, Table 1)
and on the Tiago arm; neither is available, so these generators stand in for
them at the paper's map shapes (Table 1: 192/256/512 x 128 voxels at
0.5/1/2 cm) with a synthetic 7-DoF arm.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------------------
# plain occupancy grids
# ---------------------------------------------------------------------------


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_grid(shape, density: float, seed: int) -> np.ndarray:
    """uint8 grid of shape (nz, ny, nx), each voxel occupied with prob. density."""
    g = rng(seed)
    return (g.random(shape) < density).astype(np.uint8)


def boxes_grid(n: int = 64, density: float = 0.02, n_boxes: int = 4,
               side_lo: int = 4, side_hi: int = 12, seed: int = 0) -> np.ndarray:
    """n^3 grid: Bernoulli(density) voxels plus n_boxes axis-aligned boxes.

    Box side per axis is uniform in {side_lo..side_hi}; the min corner is
    uniform over positions where the box fits inside the grid.
    """
    g = rng(seed)
    occ = (g.random((n, n, n)) < density).astype(np.uint8)
    for _ in range(n_boxes):
        s = g.integers(side_lo, side_hi + 1, size=3)
        c = np.array([g.integers(0, n - int(si) + 1) for si in s])
        occ[c[2]:c[2] + s[2], c[1]:c[1] + s[1], c[0]:c[0] + s[0]] = 1
    return occ


def blobs_grid(n: int = 512, frac: float = 0.05, sigma: float = 3.0,
               pts_per_blob: int = 256, seed: int = 0, nz: int | None = None,
               ny: int | None = None) -> np.ndarray:
    """Clustered-blob occupancy with exactly round(frac * N) occupied voxels.

    Cluster centres are uniform in the grid (a Poisson process conditioned on
    the count); each blob draws pts_per_blob voxel offsets ~ N(0, sigma^2)
    per axis, rounded.  Blobs are added in order until the number of distinct
    occupied voxels reaches the target; the last blob is trimmed so the count
    is exact.
    """
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    total = nx * ny * nz
    target = int(round(frac * total))
    g = rng(seed)
    occ = np.zeros(total, dtype=np.uint8)
    have = 0
    batch = 4096
    while have < target:
        cen = g.random((batch, 3)) * np.array([nx, ny, nz])
        off = np.rint(g.normal(0.0, sigma, size=(batch, pts_per_blob, 3)))
        p = np.floor(cen)[:, None, :] + off
        p = p.reshape(-1, 3)
        ok = ((p[:, 0] >= 0) & (p[:, 0] < nx) & (p[:, 1] >= 0) & (p[:, 1] < ny)
              & (p[:, 2] >= 0) & (p[:, 2] < nz))
        lin = (p[:, 0] + nx * (p[:, 1] + ny * p[:, 2])).astype(np.int64)
        lin = lin[ok]
        lin = lin[occ[lin] == 0]
        # first occurrence of each new voxel, in generation order
        uniq, first = np.unique(lin, return_index=True)
        order = np.sort(first)
        new = lin[order]
        need = target - have
        if new.size > need:
            new = new[:need]
        occ[new] = 1
        have += new.size
    return occ.reshape(nz, ny, nx)


def single_site_grid(shape, site_xyz) -> np.ndarray:
    occ = np.zeros(shape, dtype=np.uint8)
    x, y, z = site_xyz
    occ[z, y, x] = 1
    return occ


# ---------------------------------------------------------------------------
# map geometry
# ---------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Grid:
    """Regular voxel grid; x is the fastest memory axis (lin = x + nx*(y + ny*z))."""
    nx: int
    ny: int
    nz: int
    origin: tuple = (0.0, 0.0, 0.0)   # metres, min corner of voxel (0,0,0)
    voxel: float = 0.01               # metres

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    @property
    def extent(self):
        return (self.nx * self.voxel, self.ny * self.voxel, self.nz * self.voxel)


# ---------------------------------------------------------------------------
# rigid transforms (input preparation: sensor pose, link poses)
# ---------------------------------------------------------------------------


def rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def pose12(R, t) -> np.ndarray:
    """Row-major 3x4 [R | t] as float32[12]."""
    return np.concatenate([np.hstack([np.asarray(R, np.float64),
                                      np.asarray(t, np.float64).reshape(3, 1)]).reshape(-1)]
                          ).astype(np.float32)


# ---------------------------------------------------------------------------
# synthetic depth camera (stands in for the paper's 30 Hz Xtion point cloud)
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Camera:
    width: int = 640
    height: int = 480
    fx: float = 525.0
    fy: float = 525.0
    cx: float = 319.5
    cy: float = 239.5
    position: tuple = (1.28, -0.4, 1.0)
    pitch_deg: float = 25.0       # downward tilt from horizontal, looking along +y

    def R_map_cam(self) -> np.ndarray:
        # optical frame: z forward, x right, y down.  Forward = +y of the map,
        # right = +x, down = -z, then pitch down about the camera's x axis.
        base = np.array([[1.0, 0.0, 0.0],
                         [0.0, 0.0, 1.0],
                         [0.0, -1.0, 0.0]])
        p = math.radians(self.pitch_deg)
        # pitching forward-down: rotate the optical frame about its own x axis
        return base @ rot_x(-p)

    def T_map_cam(self) -> np.ndarray:
        return pose12(self.R_map_cam(), self.position)


@dataclasses.dataclass
class Scene:
    boxes: list        # (centre[3], half[3], yaw)
    spheres: list      # (centre[3], radius)
    mover: tuple       # (start[3], velocity[3], radius)
    floor_z: float
    wall_y: float
    lo: np.ndarray
    hi: np.ndarray

    def mover_at(self, t: float) -> np.ndarray:
        """Straight-line motion reflecting at the workspace bounds."""
        p0, v, r = self.mover
        p = np.array(p0, dtype=np.float64) + np.array(v) * t
        lo = self.lo + r
        hi = self.hi - r
        span = hi - lo
        q = np.mod(p - lo, 2 * span)
        q = np.where(q > span, 2 * span - q, q)
        return lo + q


def make_scene(grid: Grid, seed: int) -> Scene:
    g = rng(seed)
    ext = np.array(grid.extent)
    # workspace: the map minus margins proportional to its extent
    lo = np.array(grid.origin) + ext * np.array([0.08, 0.16, 0.08])
    hi = np.array(grid.origin) + ext * np.array([0.92, 0.88, 0.92])
    boxes = []
    for _ in range(5):
        side = g.uniform(0.05, 0.30, size=3)
        c = g.uniform(lo, hi)
        boxes.append((c, side / 2, g.uniform(0, 2 * math.pi)))
    spheres = []
    for _ in range(5):
        spheres.append((g.uniform(lo, hi), g.uniform(0.05, 0.15)))
    d = g.normal(size=3)
    d /= np.linalg.norm(d)
    r_mov = min(0.10, 0.25 * float(np.min(hi - lo)))
    mover = (g.uniform(lo + r_mov, hi - r_mov), 1.5 * d, r_mov)
    return Scene(boxes, spheres, mover, floor_z=grid.origin[2] + 0.05,
                 wall_y=grid.origin[1] + ext[1] - 0.06, lo=lo, hi=hi)


def _ray_sphere(o, d, c, r):
    oc = o - c
    b = d @ oc
    cc = oc @ oc - r * r
    disc = b * b - cc
    t = -b - np.sqrt(np.maximum(disc, 0.0))
    return np.where((disc >= 0) & (t > 1e-6), t, np.inf)


def _ray_box(o, d, c, half, yaw):
    Rz = rot_z(yaw)
    ol = (o - c) @ Rz          # into box frame: R^T (o - c)
    dl = d @ Rz
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dl
        t1 = (-half - ol) * inv
        t2 = (half - ol) * inv
    tmin = np.nanmax(np.minimum(t1, t2), axis=-1)
    tmax = np.nanmin(np.maximum(t1, t2), axis=-1)
    hit = (tmax >= tmin) & (tmax > 1e-6)
    t = np.where(tmin > 1e-6, tmin, tmax)
    return np.where(hit, t, np.inf)


def depth_frame(cam: Camera, scene: Scene, frame: int, seed: int,
                noise_sigma: float = 0.005) -> np.ndarray:
    """Ray-cast one frame; returns float32 points [H*W, 3] in the camera frame.

    Every pixel hits something (floor plane or back wall close the scene);
    depth along the optical axis gets N(0, noise_sigma^2) additive noise.
    Points that land outside the map are kept: insertion drops them.
    """
    g = rng(seed * 1000003 + frame)
    u, v = np.meshgrid(np.arange(cam.width), np.arange(cam.height))
    dirs_cam = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy,
                         np.ones_like(u, dtype=np.float64)], -1).reshape(-1, 3)
    R = cam.R_map_cam()
    o = np.array(cam.position, dtype=np.float64)
    d = dirs_cam @ R.T                      # map-frame ray, |d_z_cam| = 1
    t = np.full(d.shape[0], np.inf)
    # floor z = floor_z
    with np.errstate(divide="ignore", invalid="ignore"):
        tf = (scene.floor_z - o[2]) / d[:, 2]
        tw = (scene.wall_y - o[1]) / d[:, 1]
    t = np.minimum(t, np.where(tf > 0, tf, np.inf))
    t = np.minimum(t, np.where(tw > 0, tw, np.inf))
    for c, half, yaw in scene.boxes:
        t = np.minimum(t, _ray_box(o, d, np.asarray(c), np.asarray(half), yaw))
    for c, r in scene.spheres:
        t = np.minimum(t, _ray_sphere(o, d, np.asarray(c), r))
    t = np.minimum(t, _ray_sphere(o, d, scene.mover_at(frame / 30.0), scene.mover[2]))
    t = np.where(np.isfinite(t), t, 10.0)
    # t is the depth along the optical axis because dirs_cam has unit z
    t = t + g.normal(0.0, noise_sigma, size=t.shape)
    pts = dirs_cam * t[:, None]
    return pts.astype(np.float32)


# ---------------------------------------------------------------------------
# synthetic 7-DoF arm (stands in for the Tiago arm; Sec. III-A, III-B)
# ---------------------------------------------------------------------------

JOINT_AXES = "zyzyzyz"


@dataclasses.dataclass
class Robot:
    base: np.ndarray        # map-frame position of link 0's origin
    radii: np.ndarray       # [8] capsule radius per link (m)
    lengths: np.ndarray     # [8] capsule segment length per link (m)
    torso_down: bool = False  # link 0 points down from the base instead of up

    @property
    def n_links(self):
        return len(self.radii)

    def fk(self, q) -> np.ndarray:
        """Link frames for joint vector q[7]: float64 [8, 3, 4] (map frame).

        Link 0 is fixed at the base.  Joint i (1..7) sits at the far end of
        link i-1 and rotates about that frame's z or y axis (z-y-z-y-z-y-z).
        Each link's capsule runs along its local +z from 0 to its length.
        """
        q = np.asarray(q, dtype=np.float64)
        R = np.eye(3)
        if self.torso_down:
            R = rot_x(math.pi)
        t = np.asarray(self.base, dtype=np.float64).copy()
        out = np.zeros((self.n_links, 3, 4))
        out[0, :, :3] = R
        out[0, :, 3] = t
        for i in range(1, self.n_links):
            t = t + R[:, 2] * self.lengths[i - 1]
            ax = JOINT_AXES[i - 1]
            R = R @ (rot_z(q[i - 1]) if ax == "z" else rot_y(q[i - 1]))
            out[i, :, :3] = R
            out[i, :, 3] = t
        return out

    def fk_batch(self, qs) -> np.ndarray:
        """Link frames for many joint states: float64 [N, 8, 3, 4]."""
        qs = np.asarray(qs, dtype=np.float64)
        n = qs.shape[0]
        R = np.broadcast_to(rot_x(math.pi) if self.torso_down else np.eye(3), (n, 3, 3)).copy()
        t = np.broadcast_to(np.asarray(self.base, np.float64), (n, 3)).copy()
        out = np.zeros((n, self.n_links, 3, 4))
        out[:, 0, :, :3] = R
        out[:, 0, :, 3] = t
        for i in range(1, self.n_links):
            t = t + R[:, :, 2] * self.lengths[i - 1]
            a = qs[:, i - 1]
            c, s_ = np.cos(a), np.sin(a)
            J = np.zeros((n, 3, 3))
            if JOINT_AXES[i - 1] == "z":
                J[:, 0, 0], J[:, 0, 1], J[:, 1, 0], J[:, 1, 1], J[:, 2, 2] = c, -s_, s_, c, 1.0
            else:
                J[:, 0, 0], J[:, 0, 2], J[:, 2, 0], J[:, 2, 2], J[:, 1, 1] = c, s_, -s_, c, 1.0
            R = R @ J
            out[:, i, :, :3] = R
            out[:, i, :, 3] = t
        return out

    def poses12(self, q) -> np.ndarray:
        f = self.fk(q)
        return f.reshape(self.n_links, 12).astype(np.float32)

    def joint_frames(self, q):
        """(axes [7, 3], origins [7, 3]) of the joints at state q, world frame:
        joint i (1..7) sits at the origin of link i and turns about that
        frame's z or y axis; a point on link L is moved by joints 1..L."""
        f = self.fk(q)
        axes = np.array([f[i + 1][:, 2] if JOINT_AXES[i] == "z" else f[i + 1][:, 1]
                         for i in range(len(JOINT_AXES))])
        origins = np.array([f[i + 1][:, 3] for i in range(len(JOINT_AXES))])
        return axes, origins


def make_robot(seed: int, base=(1.28, 1.28, 0.3), r_lo=0.04, r_hi=0.08,
               l_lo=0.20, l_hi=0.40, torso_down=False) -> Robot:
    g = rng(seed)
    return Robot(base=np.asarray(base, dtype=np.float64),
                 radii=g.uniform(r_lo, r_hi, size=8),
                 lengths=g.uniform(l_lo, l_hi, size=8),
                 torso_down=torso_down)


def compact_robot(seed: int, base=(0.64, 0.64, 0.64)) -> Robot:
    """Arm whose full reach fits a 128^3 map at 1 cm centred on its base:
    8 links of at most 7.5 cm plus a sphere overhang stay within 0.64 m."""
    return make_robot(seed, base=base, r_lo=0.02, r_hi=0.035, l_lo=0.05,
                      l_hi=0.075, torso_down=True)


def random_joint_states(n: int, seed: int, limit_deg: float = 170.0) -> np.ndarray:
    g = rng(seed)
    lim = math.radians(limit_deg)
    return g.uniform(-lim, lim, size=(n, 7))


def capsule_lattice(radius: float, length: float, voxel: float) -> np.ndarray:
    """Points of a half-voxel cubic lattice inside a capsule (link frame).

    Stands in for the offline mesh voxelization of Sec. III-A: the capsule is
    the segment [0, length] on +z swept by a ball of the given radius.  The
    lattice spacing is voxel/2, whose covering radius (0.433 voxel) is below
    half a voxel, so every voxel whose inscribed ball lies inside the capsule
    receives at least one point at any pose.
    """
    s = voxel / 2.0
    k = int(math.ceil(radius / s)) + 1
    kz0 = -k
    kz1 = int(math.ceil((length + radius) / s)) + 1
    ax = np.arange(-k, k + 1) * s
    az = np.arange(kz0, kz1 + 1) * s
    X, Y, Z = np.meshgrid(ax, ax, az, indexing="ij")
    zc = np.clip(Z, 0.0, length)
    dd = X * X + Y * Y + (Z - zc) ** 2
    m = dd <= radius * radius
    return np.stack([X[m], Y[m], Z[m]], -1).astype(np.float32)


def link_models(robot: Robot, voxel: float):
    """(points float32 [P,3], offsets int32 [L+1]) for all links."""
    pts = [capsule_lattice(float(r), float(l), voxel)
           for r, l in zip(robot.radii, robot.lengths)]
    off = np.zeros(len(pts) + 1, dtype=np.int32)
    off[1:] = np.cumsum([p.shape[0] for p in pts])
    return np.concatenate(pts, 0), off


def bounding_spheres_link(radius: float, length: float):
    """OBB-aligned bounding spheres of one capsule link (Sec. III-B).

    The capsule's OBB has edges d1 = d2 = 2r and d3 = length + 2r.  Sphere
    diameter is sqrt(d1^2 + d2^2); the count is ceil(d3 / diameter + 1);
    centres are spaced evenly along the long axis from one end of the box to
    the other.  Returns (centres in link frame [k,3], radii [k]).
    """
    d1 = d2 = 2.0 * radius
    d3 = length + 2.0 * radius
    dia = math.sqrt(d1 * d1 + d2 * d2)
    k = int(math.ceil(d3 / dia + 1.0))
    zs = np.linspace(-radius, length + radius, k)
    c = np.zeros((k, 3))
    c[:, 2] = zs
    return c, np.full(k, dia / 2.0)


def sphere_set(robot: Robot, links, max_spheres: int):
    """Sphere (link index, centre in link frame, radius) on the given links."""
    li, cs, rs = [], [], []
    for l in links:
        c, r = bounding_spheres_link(float(robot.radii[l]), float(robot.lengths[l]))
        li += [l] * len(r)
        cs.append(c)
        rs.append(r)
    li = np.array(li[:max_spheres], dtype=np.int32)
    cs = np.concatenate(cs, 0)[:max_spheres]
    rs = np.concatenate(rs, 0)[:max_spheres]
    return li, cs, rs


def sphere_centres(robot: Robot, q, links_idx, centres_link) -> np.ndarray:
    """Map-frame sphere centres for joint state q (forward kinematics)."""
    f = robot.fk(q)
    out = np.einsum("kij,kj->ki", f[links_idx, :, :3], centres_link) + f[links_idx, :, 3]
    return out.astype(np.float32)


# ---------------------------------------------------------------------------
# control-cycle workload (256 x 256 x 128 at 1 cm)
# ---------------------------------------------------------------------------

CYCLE_GRID = Grid(256, 256, 128, (0.0, 0.0, 0.0), 0.01)


@dataclasses.dataclass
class CycleInputs:
    grid: Grid
    frames: list            # float32 [n_pts, 3] camera-frame clouds
    T_map_cam: np.ndarray   # float32 [12]
    link_pts: np.ndarray    # float32 [P, 3]
    link_off: np.ndarray    # int32 [L+1]
    robot: Robot
    sphere_links: np.ndarray
    sphere_local: np.ndarray
    sphere_radii: np.ndarray
    joint_states: np.ndarray  # float64 [n_cycles, 7]


def with_outliers(points: np.ndarray, frac: float, seed: int, nan_frac: float = 0.0) -> np.ndarray:
    """Copy of a camera-frame cloud in which a fraction frac of the points are
    moved along their own ray to a random 30-90% of their depth (the flying
    pixels of depth cameras) and a fraction nan_frac become NaN (no return)."""
    g = rng(seed)
    out = np.array(points, np.float32, copy=True)
    n = out.shape[0]
    idx = g.choice(n, int(round(frac * n)), replace=False)
    out[idx] *= g.uniform(0.3, 0.9, (idx.size, 1)).astype(np.float32)
    if nan_frac > 0:
        out[g.choice(n, int(round(nan_frac * n)), replace=False)] = np.nan
    return out


def cycle_inputs(seed: int = 0, n_frames: int = 4, n_states: int = 16,
                 grid: Grid = CYCLE_GRID) -> CycleInputs:
    cam = Camera()
    scene = make_scene(grid, seed)
    frames = [depth_frame(cam, scene, k, seed) for k in range(n_frames)]
    robot = make_robot(seed + 1)
    lp, lo = link_models(robot, grid.voxel)
    li, cs, rs = sphere_set(robot, range(1, 8), 20)
    return CycleInputs(grid, frames, cam.T_map_cam(), lp, lo, robot, li, cs,
                       rs.astype(np.float32), random_joint_states(n_states, seed + 2))


# ---------------------------------------------------------------------------
# batched workload: many maps of uneven size, each with its own scene
# ---------------------------------------------------------------------------


def batch_grids(n_maps: int, seed: int, lo=(64, 64, 64), hi=(256, 256, 128),
                voxel: float = 0.01) -> list:
    """Grids with every axis uniform in [lo, hi] (ragged, not rounded)."""
    g = rng(seed)
    out = []
    for _ in range(n_maps):
        nx, ny, nz = (int(g.integers(lo[i], hi[i] + 1)) for i in range(3))
        out.append(Grid(nx, ny, nz, (0.0, 0.0, 0.0), voxel))
    return out


@dataclasses.dataclass
class BatchInputs:
    grids: list
    clouds: list              # float32 [n_m, 3] camera frame, one per map
    T_map_cam: list           # float32 [12] per map
    robots: list              # Robot per map (compact arm at the map centre)
    lookahead: list           # float64 [S, 7] joint states per map
    sphere_links: np.ndarray  # spheres on links 4..7 (shared layout)
    sphere_local: list        # per map: centres in link frames
    sphere_radii: list        # per map: float32 [m]
    centres: list             # per map: float32 [S, m, 3] map-frame centres


def batch_inputs(seed: int = 0, n_maps: int = 32, n_states: int = 16, min_points: int = 50_000,
                 max_points: int = 300_000, n_spheres: int = 20, grids=None) -> BatchInputs:
    """Batched cycle: per map its own depth frame subsampled to a point count
    uniform in [min_points, max_points], an arm at the map centre, and
    n_states look-ahead joint states q + U[-0.1, 0.1] rad per joint."""
    g = rng(seed)
    grids = grids if grids is not None else batch_grids(n_maps, seed)
    clouds, Ts, robots, look, locs, rads, cents = [], [], [], [], [], [], []
    li = None
    for m, grid in enumerate(grids):
        ext = np.array(grid.extent)
        cam = Camera(position=(ext[0] / 2, -0.4, 0.78 * ext[2]))
        scene = make_scene(grid, seed * 1000 + m)
        pts = depth_frame(cam, scene, 0, seed * 1000 + m)
        k = int(g.integers(min_points, max_points + 1))
        sel = np.sort(g.choice(pts.shape[0], size=min(k, pts.shape[0]), replace=False))
        clouds.append(np.ascontiguousarray(pts[sel]))
        Ts.append(cam.T_map_cam())
        robot = compact_robot(seed * 1000 + m, base=tuple(ext / 2))
        robots.append(robot)
        q0 = random_joint_states(1, seed * 1000 + m)[0]
        qs = q0[None, :] + g.uniform(-0.1, 0.1, size=(n_states, 7))
        look.append(qs)
        li, cs, rs = sphere_set(robot, range(1, 8), n_spheres)
        locs.append(cs)
        rads.append(rs.astype(np.float32))
        cents.append(np.stack([sphere_centres(robot, q, li, cs) for q in qs]))
    return BatchInputs(grids, clouds, Ts, robots, look, li, locs, rads, cents)


# ---------------------------------------------------------------------------
# learned self-distance surrogate: self-map workload
# ---------------------------------------------------------------------------

SELF_GRID = Grid(128, 128, 128, (0.0, 0.0, 0.0), 0.01)
SELF_OBSTACLE_MASK = 0b0000_0011     # torso (link 0) and shoulder (link 1)
SELF_SPHERE_LINKS = (4, 5, 6, 7)
SELF_N_SPHERES = 12


@dataclasses.dataclass
class SelfMapSetup:
    grid: Grid
    robot: Robot
    link_pts: np.ndarray
    link_off: np.ndarray
    mask: int
    sphere_links: np.ndarray
    sphere_local: np.ndarray
    sphere_radii: np.ndarray


def self_map_robot() -> Robot:
    """The arm of the self-collision workload: a thick torso (link 0, 25 cm
    long, 10 cm radius) rising from (0.64, 0.64, 0.35) m, a short shoulder
    and six arm links.  From the shoulder at z = 0.60 m its whole reach,
    sphere overhang included (0.595 m), stays inside the 1.28 m map."""
    return Robot(base=np.array([0.64, 0.64, 0.35]),
                 radii=np.array([0.10, 0.05, 0.04, 0.035, 0.03, 0.03, 0.025, 0.025]),
                 lengths=np.array([0.25, 0.06, 0.12, 0.10, 0.10, 0.08, 0.06, 0.05]))


def self_map_setup() -> SelfMapSetup:
    """128^3 map at 1 cm around the arm, obstacle links 0-1 (the links not
    in the allowed-collision set of the distal arm, Eq. selfclink) and 12
    bounding spheres on links 4-7 (Sec. III-B rule, 3 per link)."""
    g = SELF_GRID
    robot = self_map_robot()
    lp, lo = link_models(robot, g.voxel)
    li, cs, rs = sphere_set(robot, SELF_SPHERE_LINKS, SELF_N_SPHERES)
    assert len(rs) == SELF_N_SPHERES
    return SelfMapSetup(g, robot, lp, lo, SELF_OBSTACLE_MASK, li, cs, rs.astype(np.float32))


def sphere_centres_batch(robot: Robot, qs, links_idx, centres_link) -> np.ndarray:
    """float32 [N, m, 3] map-frame sphere centres for many joint states."""
    f = robot.fk_batch(qs)
    fl = f[:, links_idx]          # [N, m, 3, 4]
    R = fl[..., :3]
    t = fl[..., 3]
    return (np.einsum("nkij,kj->nki", R, centres_link) + t).astype(np.float32)
