"""CPU oracle for the distance-map hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library: the C file
``edt_ref.c`` is built here with gcc into ``liboracle.so``, and ``brute``
holds an independent all-pairs reference used to pin it.

Functions (each cites the paper passage it follows in its docstring):
  edt(occ)              exact squared EDT + nearest-site index (Sec. III-C)
  insert_points(...)    point-cloud insertion (Sec. III-A)
  insert_links(...)     link voxel models placed by joint state (Sec. III-A)
  query_spheres(...)    closest obstacle at sphere centres (Alg. 2, Eq. dist)
  update_logodds(...)   per-frame Bayesian occupancy update (Sec. III-A)
  ray_walk(a, b)        voxels a sensor ray crosses (the update's traversal)
  outlier_filter(...)   statistical outlier filtering of a cloud (Sec. III-A)
  jfa(occ)              jump flooding, the approximate transform of Table 2
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "edt_ref.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

QUERY_WORDS = 16     # 4-byte words per sphere result
Q_OUT_OF_MAP = 1
Q_EMPTY = 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O3, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_edt.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int]
        lib.oracle_edt.restype = ctypes.c_int
        lib.oracle_insert_points.argtypes = [ctypes.c_int] * 3 + [P, ctypes.c_float, P, P,
                                                                   ctypes.c_int64, P, P]
        lib.oracle_insert_points.restype = None
        lib.oracle_insert_links.argtypes = [ctypes.c_int] * 3 + [P, ctypes.c_float, P, P, P,
                                                                  ctypes.c_int, P, ctypes.c_uint64]
        lib.oracle_insert_links.restype = None
        lib.oracle_query_spheres.argtypes = [ctypes.c_int] * 3 + [P, ctypes.c_float, P, P, P, P,
                                                                   ctypes.c_int, P]
        lib.oracle_query_spheres.restype = None
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_ray_walk.argtypes = [P, P, P, ctypes.c_int]
        lib.oracle_ray_walk.restype = ctypes.c_int
        lib.oracle_update_logodds.argtypes = ([ctypes.c_int] * 3 + [P, ctypes.c_float, P, P, P,
                                              ctypes.c_int64, P, P, P] + [ctypes.c_int] * 5)
        lib.oracle_update_logodds.restype = None
        lib.oracle_outlier_filter.argtypes = [P, ctypes.c_int64, ctypes.c_int, ctypes.c_float,
                                              ctypes.c_double, P, P, P]
        lib.oracle_outlier_filter.restype = None
        lib.oracle_outlier_mean_dist.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int,
                                                 ctypes.c_float, P]
        lib.oracle_outlier_mean_dist.restype = None
        lib.oracle_jfa.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        lib.oracle_jfa.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def edt(occ: np.ndarray, nthreads: int = 0):
    """Exact squared EDT of an occupancy grid [nz, ny, nx] (Sec. III-C, Alg. 1).

    Returns (d2 int32, site int32) of the same shape; site is the linear index
    x + nx*(y + ny*z) of the nearest occupied voxel, the smallest such index
    on ties; an empty grid gives INT32_MAX / -1 everywhere.
    """
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    nz, ny, nx = occ.shape
    d2 = np.empty(occ.shape, np.int32)
    site = np.empty(occ.shape, np.int32)
    rc = _load().oracle_edt(_ptr(occ), nx, ny, nz, _ptr(d2), _ptr(site), int(nthreads))
    if rc != 0:
        raise RuntimeError("oracle_edt failed")
    return d2, site


def _grid_args(grid):
    origin = np.asarray(grid.origin, np.float32)
    return grid.nx, grid.ny, grid.nz, origin, np.float32(grid.voxel)


def insert_points(grid, occ: np.ndarray, pts: np.ndarray, T: np.ndarray,
                  exclude: np.ndarray | None = None) -> np.ndarray:
    """OR a point cloud into occ (Sec. III-A); returns occ (modified in place)."""
    nx, ny, nz, origin, v = _grid_args(grid)
    pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 3)
    T = np.ascontiguousarray(T, np.float32).reshape(12)
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous and occ.size == grid.n
    ex = None if exclude is None else np.ascontiguousarray(exclude, np.uint8)
    _load().oracle_insert_points(nx, ny, nz, _ptr(origin), v, _ptr(occ), _ptr(pts),
                                 pts.shape[0], _ptr(T), None if ex is None else _ptr(ex))
    return occ


def insert_links(grid, occ: np.ndarray, link_pts: np.ndarray, link_off: np.ndarray,
                 poses: np.ndarray, mask: int) -> np.ndarray:
    """OR the masked links' voxel models, placed by their poses (Sec. III-A)."""
    nx, ny, nz, origin, v = _grid_args(grid)
    lp = np.ascontiguousarray(link_pts, np.float32).reshape(-1, 3)
    lo = np.ascontiguousarray(link_off, np.int32)
    ps = np.ascontiguousarray(poses, np.float32).reshape(-1, 12)
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous and occ.size == grid.n
    _load().oracle_insert_links(nx, ny, nz, _ptr(origin), v, _ptr(occ), _ptr(lp), _ptr(lo),
                                lo.size - 1, _ptr(ps), ctypes.c_uint64(mask))
    return occ


def query_spheres(grid, d2: np.ndarray, site: np.ndarray, centres: np.ndarray,
                  radii: np.ndarray) -> np.ndarray:
    """Closest-obstacle query at sphere centres (Alg. 2; Eq. dist).

    Returns uint32 [m, 16]: d2, site, voxel[3], flags, dist_vox, x_c,
    clearance, grad[3], nearest[3], 0 (floats as raw bits).
    """
    nx, ny, nz, origin, v = _grid_args(grid)
    c = np.ascontiguousarray(centres, np.float32).reshape(-1, 3)
    r = np.ascontiguousarray(radii, np.float32).reshape(-1)
    d2 = np.ascontiguousarray(d2, np.int32)
    site = np.ascontiguousarray(site, np.int32)
    out = np.zeros((c.shape[0], QUERY_WORDS), np.uint32)
    _load().oracle_query_spheres(nx, ny, nz, _ptr(origin), v, _ptr(d2), _ptr(site), _ptr(c),
                                 _ptr(r), c.shape[0], _ptr(out))
    return out


def ray_walk(a, b) -> np.ndarray:
    """Voxels (int32 [k, 3]) the ray from a to b (voxel units) crosses, from
    floor(a) to floor(b), one voxel per step (Amanatides-Woo order)."""
    a = np.ascontiguousarray(a, np.float32).reshape(3)
    b = np.ascontiguousarray(b, np.float32).reshape(3)
    cap = int(np.abs(np.floor(b) - np.floor(a)).sum()) + 1
    out = np.zeros((cap, 3), np.int32)
    steps = _load().oracle_ray_walk(_ptr(a), _ptr(b), _ptr(out), cap)
    assert steps + 1 == cap
    return out


# log-odds parameters in hundredths of a nat: P(hit) 0.7, P(miss) 0.4,
# clamped to [-2.0, 3.5], occupied above 0 (probability above one half)
LOGODDS_DEFAULT = dict(hit=85, miss=-41, lmin=-200, lmax=350, threshold=0)


def update_logodds(grid, logodds: np.ndarray, occ: np.ndarray, pts: np.ndarray, T: np.ndarray,
                   exclude: np.ndarray | None = None, hit=85, miss=-41, lmin=-200, lmax=350,
                   threshold=0, keep: np.ndarray | None = None):
    """One frame's Bayesian occupancy update (Sec. III-A), in place on the
    int16 log-odds grid; occ (uint8) becomes logodds > threshold."""
    nx, ny, nz, origin, v = _grid_args(grid)
    pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 3)
    T = np.ascontiguousarray(T, np.float32).reshape(12)
    assert logodds.dtype == np.int16 and logodds.flags.c_contiguous and logodds.size == grid.n
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous and occ.size == grid.n
    ex = None if exclude is None else np.ascontiguousarray(exclude, np.uint8)
    kp = None if keep is None else np.ascontiguousarray(keep, np.uint8)
    assert kp is None or kp.size == pts.shape[0]
    _load().oracle_update_logodds(nx, ny, nz, _ptr(origin), v, _ptr(logodds), _ptr(occ), _ptr(pts),
                                  pts.shape[0], _ptr(T), None if kp is None else _ptr(kp),
                                  None if ex is None else _ptr(ex),
                                  int(hit), int(miss), int(lmin), int(lmax), int(threshold))
    return logodds, occ


def outlier_filter(pts: np.ndarray, k: int = 8, radius: float = 0.01, alpha: float = 1.0):
    """Statistical outlier filtering (Sec. III-A): (keep uint8 [n], mean
    neighbour distance float32 [n] (NaN for non-finite points), (mu, sigma,
    threshold)).  Brute force over all pairs: O(n^2)."""
    pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 3)
    n = pts.shape[0]
    assert 1 <= k <= 64
    keep = np.zeros(n, np.uint8)
    dm = np.zeros(n, np.float32)
    stats = np.zeros(3, np.float64)
    _load().oracle_outlier_filter(_ptr(pts), n, int(k), float(radius), float(alpha), _ptr(keep),
                                  _ptr(dm), _ptr(stats))
    return keep, dm, tuple(float(x) for x in stats)


def outlier_mean_dist(pts: np.ndarray, idx: np.ndarray, k: int = 8, radius: float = 0.01):
    """The outlier filter's mean neighbour distance d_i for the listed points
    only (same definition as outlier_filter, O(len(idx) * n))."""
    pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 3)
    idx = np.ascontiguousarray(idx, np.int64)
    out = np.zeros(idx.size, np.float32)
    _load().oracle_outlier_mean_dist(_ptr(pts), pts.shape[0], _ptr(idx), idx.size, int(k),
                                     float(radius), _ptr(out))
    return out


def jfa(occ: np.ndarray):
    """Jump flooding (the approximate transform compared in Table 2): (d2,
    site) like edt(), but each voxel's site is only the best the flooding
    found."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    nz, ny, nx = occ.shape
    d2 = np.empty(occ.shape, np.int32)
    site = np.empty(occ.shape, np.int32)
    if _load().oracle_jfa(_ptr(occ), nx, ny, nz, _ptr(d2), _ptr(site)) != 0:
        raise RuntimeError("oracle_jfa failed")
    return d2, site
