"""Thin ctypes binding of libedtmi.so (declared in include/edt.h).

Argument marshalling only: every function forwards device pointers of torch
tensors and the current HIP stream to the C entry point of the same name and
raises EdtError on a negative status.  All compute runs in the library's HIP
kernels; if the library is missing the first call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libedtmi.so")
_lib = None

INT32_MAX = 2 ** 31 - 1
Q_OUT_OF_MAP = 1
Q_EMPTY = 2


class EdtError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class EdtGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("origin", ctypes.c_float * 3), ("voxel", ctypes.c_float)]


class SphereResult(ctypes.Structure):
    _fields_ = [("d2", ctypes.c_int32), ("site", ctypes.c_int32), ("vox", ctypes.c_int32 * 3),
                ("flags", ctypes.c_int32), ("dist_vox", ctypes.c_float), ("x_c", ctypes.c_float),
                ("clearance", ctypes.c_float), ("grad", ctypes.c_float * 3),
                ("nearest", ctypes.c_float * 3), ("reserved", ctypes.c_float)]


class Tuning(ctypes.Structure):
    _fields_ = [("xy_tile", ctypes.c_int32), ("z_tile", ctypes.c_int32), ("z_group", ctypes.c_int32),
                ("xy_group", ctypes.c_int32)]


class LogOdds(ctypes.Structure):
    _fields_ = [("hit", ctypes.c_int16), ("miss", ctypes.c_int16), ("min", ctypes.c_int16),
                ("max", ctypes.c_int16), ("threshold", ctypes.c_int16), ("reserved", ctypes.c_int16)]


# hundredths of a nat: P(hit) 0.7, P(miss) 0.4, clamp [-2.0, 3.5], occupied above 0
LOGODDS_DEFAULT = (85, -41, -200, 350, 0)


class BatchMap(ctypes.Structure):
    _fields_ = [("grid", EdtGrid), ("occ", ctypes.c_void_p), ("d2", ctypes.c_void_p),
                ("site", ctypes.c_void_p)]


SPHERE_RESULT_BYTES = ctypes.sizeof(SphereResult)   # 64
SPHERE_RESULT_WORDS = SPHERE_RESULT_BYTES // 4

EXPORTED = ["edt_status_string", "edt_last_error", "edt_version", "edt_clear",
            "edt_insert_points", "edt_insert_links", "edt_workspace_bytes", "edt_compute",
            "edt_query_spheres", "edt_compute_stage", "edt_default_tuning", "edt_compute_tuned",
            "edt_autotune", "edt_batch_workspace_bytes", "edt_compute_batched", "edt_batch_status",
            "edt_compute_many", "edt_logodds_workspace_bytes", "edt_logodds_reset",
            "edt_update_logodds", "edt_outlier_workspace_bytes", "edt_outlier_filter",
            "edt_cache_workspace_bytes", "edt_cache_reset", "edt_compute_cached",
            "edt_jfa_workspace_bytes", "edt_jfa",
            "edt_autotune_batched", "edt_compute_batched_noalloc", "edt_compute_many_gated",
            "edt_clear_insert_links_many", "edt_query_spheres_many", "edt_clear_insert_points_many",
            "edt_tuning_cache_save",
            "edt_tuning_cache_load", "edt_tuning_cache_clear"]

BATCH_MAX = 48

STAGE_XY, STAGE_Z, STAGE_ALL = 1, 2, 3


def lib():
    """Load libedtmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_2407_02363_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, G = ctypes.c_void_p, ctypes.POINTER(EdtGrid)
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "edt_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "edt_last_error": ([], ctypes.c_char_p),
        "edt_version": ([], ctypes.c_char_p),
        "edt_clear": ([G, P, P], ctypes.c_int),
        "edt_insert_points": ([G, P, P, i64, P, P, P], ctypes.c_int),
        "edt_insert_links": ([G, P, P, P, i32, P, u64, P], ctypes.c_int),
        "edt_workspace_bytes": ([G], ctypes.c_size_t),
        "edt_compute": ([G, P, P, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "edt_query_spheres": ([G, P, P, P, P, i32, P, P], ctypes.c_int),
        "edt_clear_insert_links_many": ([G, P, i32, P, P, i32, P, u64, P, P], ctypes.c_int),
        "edt_query_spheres_many": ([P, i32, P, P, P, P, P], ctypes.c_int),
        "edt_clear_insert_points_many": ([G, P, i32, P, P, P, P], ctypes.c_int),
        "edt_tuning_cache_save": ([ctypes.c_char_p], ctypes.c_int),
        "edt_tuning_cache_load": ([ctypes.c_char_p], ctypes.c_int),
        "edt_tuning_cache_clear": ([], ctypes.c_int),
        "edt_compute_stage": ([G, P, P, P, ctypes.c_int, ctypes.POINTER(Tuning), P], ctypes.c_int),
        "edt_default_tuning": ([G, ctypes.POINTER(Tuning)], ctypes.c_int),
        "edt_compute_tuned": ([G, P, P, P, ctypes.POINTER(Tuning), P], ctypes.c_int),
        "edt_autotune": ([G, P, P, P, i32, ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_float), P],
                         ctypes.c_int),
        "edt_batch_workspace_bytes": ([i32], ctypes.c_size_t),
        "edt_compute_batched": ([P, i32, P, ctypes.c_size_t, ctypes.POINTER(Tuning), P], ctypes.c_int),
        "edt_compute_many": ([P, i32, ctypes.POINTER(Tuning), P], ctypes.c_int),
        "edt_compute_many_gated": ([P, i32, P, ctypes.POINTER(Tuning), P], ctypes.c_int),
        "edt_compute_batched_noalloc": ([P, i32, ctypes.POINTER(Tuning), P, P], ctypes.c_int),
        "edt_logodds_workspace_bytes": ([G], ctypes.c_size_t),
        "edt_logodds_reset": ([G, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "edt_update_logodds": ([G, P, P, P, i64, P, P, P, ctypes.POINTER(LogOdds), P, ctypes.c_size_t,
                                P], ctypes.c_int),
        "edt_outlier_workspace_bytes": ([i64], ctypes.c_size_t),
        "edt_cache_workspace_bytes": ([G], ctypes.c_size_t),
        "edt_jfa_workspace_bytes": ([G], ctypes.c_size_t),
        "edt_jfa": ([G, P, P, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "edt_cache_reset": ([G, P, ctypes.c_size_t, P], ctypes.c_int),
        "edt_compute_cached": ([G, P, P, P, P, ctypes.c_size_t, P], ctypes.c_int),
        "edt_outlier_filter": ([P, i64, i32, ctypes.c_float, ctypes.c_float, P, P, P, P,
                                ctypes.c_size_t, P], ctypes.c_int),
        "edt_batch_status": ([P, ctypes.POINTER(ctypes.c_int32), P], ctypes.c_int),
        "edt_autotune_batched": ([P, i32, P, ctypes.c_size_t, i32, ctypes.POINTER(Tuning),
                                  ctypes.POINTER(ctypes.c_float), P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def make_grid(g) -> EdtGrid:
    """EdtGrid from any object with nx, ny, nz, origin, voxel."""
    if isinstance(g, EdtGrid):
        return g
    return EdtGrid(int(g.nx), int(g.ny), int(g.nz), (ctypes.c_float * 3)(*map(float, g.origin)),
                   float(g.voxel))


def _check(rc: int, where: str):
    if rc != 0:
        raise EdtError(rc, where, lib().edt_last_error().decode())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, dtype, name, numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _n(g):
    return int(g.nx) * int(g.ny) * int(g.nz)


def version() -> str:
    return lib().edt_version().decode()


def edt_clear(grid, occ, stream=None):
    g = make_grid(grid)
    _check(lib().edt_clear(ctypes.byref(g), _dev(occ, torch.uint8, "occ", _n(g)), _stream(stream)),
           "edt_clear")


def edt_insert_points(grid, occ, pts, T_map_sensor, exclude=None, stream=None):
    g = make_grid(grid)
    n = pts.shape[0] if pts.dim() == 2 else pts.numel() // 3
    _check(lib().edt_insert_points(ctypes.byref(g), _dev(occ, torch.uint8, "occ", _n(g)),
                                   _dev(pts, torch.float32, "pts", 3 * n), n,
                                   _dev(T_map_sensor, torch.float32, "T_map_sensor", 12),
                                   _dev(exclude, torch.uint8, "exclude", _n(g)), _stream(stream)),
           "edt_insert_points")


def edt_insert_links(grid, occ, link_pts, link_off, link_poses, link_mask: int, stream=None):
    g = make_grid(grid)
    off = np.ascontiguousarray(np.asarray(link_off, dtype=np.int32))
    n_links = off.size - 1
    _check(lib().edt_insert_links(ctypes.byref(g), _dev(occ, torch.uint8, "occ", _n(g)),
                                  _dev(link_pts, torch.float32, "link_pts", 3 * int(off[-1])),
                                  off.ctypes.data_as(ctypes.c_void_p), n_links,
                                  _dev(link_poses, torch.float32, "link_poses", 12 * n_links),
                                  ctypes.c_uint64(link_mask), _stream(stream)),
           "edt_insert_links")


def ptr_array(tensors, dtype, name, numel):
    """Host array of the device pointers of several tensors (for the
    entry points that take one buffer per map); the caller keeps the tensors
    alive."""
    arr = (ctypes.c_void_p * len(tensors))()
    for j, t in enumerate(tensors):
        arr[j] = _dev(t, dtype, f"{name}[{j}]", numel).value
    return arr


def edt_clear_insert_links_many(grid, occs, link_pts, link_off, link_poses, link_mask: int,
                                gates=None, stream=None):
    """Clear every map of occs (uint8 device tensors of one grid), then insert
    the links of link_mask placed by link_poses[j] (float32 device
    [n_maps, n_links, 12]) into map j; gates: None or int32 device [n_maps]."""
    g = make_grid(grid)
    off = np.ascontiguousarray(np.asarray(link_off, dtype=np.int32))
    n_links = off.size - 1
    k = len(occs)
    occ_arr = ptr_array(occs, torch.uint8, "occ", _n(g))
    _check(lib().edt_clear_insert_links_many(
        ctypes.byref(g), ctypes.cast(occ_arr, ctypes.c_void_p), k,
        _dev(link_pts, torch.float32, "link_pts", 3 * int(off[-1])),
        off.ctypes.data_as(ctypes.c_void_p), n_links,
        _dev(link_poses, torch.float32, "link_poses", 12 * n_links * k), ctypes.c_uint64(link_mask),
        _dev(gates, torch.int32, "gates", k), _stream(stream)), "edt_clear_insert_links_many")


def edt_query_spheres_many(maps, centres, radii, outs, stream=None):
    """Sphere queries of every map of a batch in one launch: maps from
    batch_maps() (grid, d2, site), and per map a float32 device [m, 3]
    centres tensor, a float32 [m] radii tensor and an int32 [m, 16] output."""
    k = len(maps)
    if not (len(centres) == len(radii) == len(outs) == k):
        raise ValueError("one centres, radii and out tensor per map")
    ms = (ctypes.c_int32 * k)()
    c_arr, r_arr, o_arr = (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)()
    for j in range(k):
        m = radii[j].numel()
        ms[j] = m
        c_arr[j] = _dev(centres[j], torch.float32, f"centres[{j}]", 3 * m).value
        r_arr[j] = _dev(radii[j], torch.float32, f"radii[{j}]", m).value
        o_arr[j] = _dev(outs[j], torch.int32, f"out[{j}]", SPHERE_RESULT_WORDS * m).value
    _check(lib().edt_query_spheres_many(ctypes.cast(maps, ctypes.c_void_p), k, ctypes.cast(c_arr, ctypes.c_void_p),
                                        ctypes.cast(r_arr, ctypes.c_void_p), ctypes.cast(ms, ctypes.c_void_p),
                                        ctypes.cast(o_arr, ctypes.c_void_p), _stream(stream)),
           "edt_query_spheres_many")


def edt_clear_insert_points_many(grids, occs, clouds, poses, stream=None):
    """Clear every map, then insert map j's cloud (float32 device [n_j, 3],
    sensor frame) placed by poses[j] (float32 device [12])."""
    k = len(grids)
    if not (len(occs) == len(clouds) == len(poses) == k):
        raise ValueError("one occupancy, cloud and pose per grid")
    g_arr = (EdtGrid * k)()
    n_arr = (ctypes.c_int64 * k)()
    o_arr, p_arr, t_arr = (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)()
    for j in range(k):
        g = make_grid(grids[j])
        g_arr[j] = g
        n = clouds[j].shape[0] if clouds[j].dim() == 2 else clouds[j].numel() // 3
        n_arr[j] = n
        o_arr[j] = _dev(occs[j], torch.uint8, f"occ[{j}]", _n(g)).value
        p_arr[j] = _dev(clouds[j], torch.float32, f"pts[{j}]", 3 * n).value
        t_arr[j] = _dev(poses[j], torch.float32, f"T[{j}]", 12).value
    _check(lib().edt_clear_insert_points_many(g_arr, ctypes.cast(o_arr, ctypes.c_void_p), k,
                                              ctypes.cast(p_arr, ctypes.c_void_p),
                                              ctypes.cast(n_arr, ctypes.c_void_p),
                                              ctypes.cast(t_arr, ctypes.c_void_p), _stream(stream)),
           "edt_clear_insert_points_many")


def edt_tuning_cache_save(path) -> int:
    """Write the autotuners' cached tiles to a text file; returns the entry count."""
    rc = lib().edt_tuning_cache_save(os.fsencode(path))
    _check(min(rc, 0), "edt_tuning_cache_save")
    return rc


def edt_tuning_cache_load(path) -> int:
    """Add a saved cache's entries; returns the entry count."""
    rc = lib().edt_tuning_cache_load(os.fsencode(path))
    _check(min(rc, 0), "edt_tuning_cache_load")
    return rc


def edt_tuning_cache_clear():
    _check(lib().edt_tuning_cache_clear(), "edt_tuning_cache_clear")


def edt_workspace_bytes(grid) -> int:
    g = make_grid(grid)
    return int(lib().edt_workspace_bytes(ctypes.byref(g)))


def edt_compute(grid, occ, d2, site, ws=None, stream=None):
    g = make_grid(grid)
    n = _n(g)
    wsb = 0 if ws is None else ws.numel() * ws.element_size()
    _check(lib().edt_compute(ctypes.byref(g), _dev(occ, torch.uint8, "occ", n),
                             _dev(d2, torch.int32, "d2", n), _dev(site, torch.int32, "site", n),
                             None if ws is None else ctypes.c_void_p(ws.data_ptr()), wsb,
                             _stream(stream)),
           "edt_compute")


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, Tuning):
        return ctypes.byref(t)
    return ctypes.byref(Tuning(int(t[0]), int(t[1]), int(t[2]) if len(t) > 2 else 0,
                               int(t[3]) if len(t) > 3 else 0))


def edt_compute_stage(grid, occ, d2, site, stage: int, tuning=None, stream=None):
    g = make_grid(grid)
    n = _n(g)
    _check(lib().edt_compute_stage(ctypes.byref(g), _dev(occ, torch.uint8, "occ", n),
                                   _dev(d2, torch.int32, "d2", n),
                                   _dev(site, torch.int32, "site", n), int(stage),
                                   _tuning(tuning), _stream(stream)),
           "edt_compute_stage")


def edt_compute_tuned(grid, occ, d2, site, tuning=None, stream=None):
    g = make_grid(grid)
    n = _n(g)
    _check(lib().edt_compute_tuned(ctypes.byref(g), _dev(occ, torch.uint8, "occ", n),
                                   _dev(d2, torch.int32, "d2", n),
                                   _dev(site, torch.int32, "site", n), _tuning(tuning),
                                   _stream(stream)),
           "edt_compute_tuned")


def edt_default_tuning(grid):
    g = make_grid(grid)
    t = Tuning()
    _check(lib().edt_default_tuning(ctypes.byref(g), ctypes.byref(t)), "edt_default_tuning")
    return (t.xy_tile, t.z_tile, t.z_group, t.xy_group)


def edt_autotune(grid, occ, d2, site, reps: int = 10, stream=None):
    """Returns ((xy_tile, z_tile, z_group), microseconds of one transform)."""
    g = make_grid(grid)
    n = _n(g)
    t = Tuning()
    us = ctypes.c_float()
    _check(lib().edt_autotune(ctypes.byref(g), _dev(occ, torch.uint8, "occ", n),
                              _dev(d2, torch.int32, "d2", n), _dev(site, torch.int32, "site", n),
                              int(reps), ctypes.byref(t), ctypes.byref(us), _stream(stream)),
           "edt_autotune")
    return (t.xy_tile, t.z_tile, t.z_group, t.xy_group), float(us.value)


def edt_query_spheres(grid, d2, site, centres, radii, out, stream=None):
    """out: int32 device tensor of shape [m, 16] (64-byte result records)."""
    g = make_grid(grid)
    m = radii.numel()
    _check(lib().edt_query_spheres(ctypes.byref(g), _dev(d2, torch.int32, "d2", _n(g)),
                                   _dev(site, torch.int32, "site", _n(g)),
                                   _dev(centres, torch.float32, "centres", 3 * m),
                                   _dev(radii, torch.float32, "radii", m), m,
                                   _dev(out, torch.int32, "out", SPHERE_RESULT_WORDS * m),
                                   _stream(stream)),
           "edt_query_spheres")


def new_query_out(m: int, device="cuda") -> torch.Tensor:
    return torch.empty((m, SPHERE_RESULT_WORDS), dtype=torch.int32, device=device)


def batch_maps(grids, occs, d2s, sites):
    """Host array of BatchMap descriptors for device tensors (kept alive by
    the caller)."""
    n = len(grids)
    arr = (BatchMap * n)()
    for i in range(n):
        g = make_grid(grids[i])
        arr[i] = BatchMap(g, _dev(occs[i], torch.uint8, "occ", _n(g)).value,
                          _dev(d2s[i], torch.int32, "d2", _n(g)).value,
                          _dev(sites[i], torch.int32, "site", _n(g)).value)
    return arr


def edt_batch_workspace_bytes(n_maps: int) -> int:
    return int(lib().edt_batch_workspace_bytes(int(n_maps)))


def new_batch_workspace(n_maps: int, device="cuda"):
    return torch.empty(edt_batch_workspace_bytes(n_maps), dtype=torch.uint8, device=device)


def edt_compute_many(maps, tuning=None, stream=None):
    """maps: result of batch_maps(); one xy and one z launch for all maps."""
    _check(lib().edt_compute_many(ctypes.cast(maps, ctypes.c_void_p), len(maps), _tuning(tuning),
                                  _stream(stream)),
           "edt_compute_many")


def edt_compute_many_gated(maps, gates, tuning=None, stream=None):
    """edt_compute_many where map i is transformed only if the int32 device
    value gates[i] is nonzero when the kernels run (else left untouched)."""
    _check(lib().edt_compute_many_gated(ctypes.cast(maps, ctypes.c_void_p), len(maps),
                                        _dev(gates, torch.int32, "gates", len(maps)),
                                        _tuning(tuning), _stream(stream)),
           "edt_compute_many_gated")


def edt_compute_batched(maps, ws, tuning=None, stream=None):
    """maps: result of batch_maps(); ws: uint8 device tensor."""
    _check(lib().edt_compute_batched(ctypes.cast(maps, ctypes.c_void_p), len(maps),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _tuning(tuning),
                                     _stream(stream)),
           "edt_compute_batched")


def edt_compute_batched_noalloc(maps, tuning=None, timed_out=None, stream=None):
    """maps: result of batch_maps(); no workspace: the library's per-GPU
    array serves the batch.  timed_out: optional int32 device tensor of one
    element, set to 1 if a wait gave up."""
    flag = None
    if timed_out is not None:
        flag = _dev(timed_out, torch.int32, "timed_out", 1)
    _check(lib().edt_compute_batched_noalloc(ctypes.cast(maps, ctypes.c_void_p), len(maps),
                                             _tuning(tuning), flag, _stream(stream)),
           "edt_compute_batched_noalloc")


def edt_batch_status(ws, stream=None) -> bool:
    """True if the last batch launch on ws gave up waiting (never expected)."""
    flag = ctypes.c_int32()
    _check(lib().edt_batch_status(ctypes.c_void_p(ws.data_ptr()), ctypes.byref(flag),
                                  _stream(stream)), "edt_batch_status")
    return bool(flag.value)


def edt_autotune_batched(maps, ws, reps: int = 5, stream=None):
    t = Tuning()
    us = ctypes.c_float()
    _check(lib().edt_autotune_batched(ctypes.cast(maps, ctypes.c_void_p), len(maps),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), int(reps),
                                      ctypes.byref(t), ctypes.byref(us), _stream(stream)),
           "edt_autotune_batched")
    return (t.xy_tile, t.z_tile), float(us.value)


def edt_logodds_workspace_bytes(grid) -> int:
    return int(lib().edt_logodds_workspace_bytes(ctypes.byref(make_grid(grid))))


def new_logodds_workspace(grid, device="cuda"):
    return torch.zeros(edt_logodds_workspace_bytes(grid), dtype=torch.uint8, device=device)


def edt_logodds_reset(grid, logodds, ws, stream=None):
    g = make_grid(grid)
    _check(lib().edt_logodds_reset(ctypes.byref(g), _dev(logodds, torch.int16, "logodds", _n(g)),
                                   _dev(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)),
           "edt_logodds_reset")


def edt_update_logodds(grid, logodds, occ, pts, T_map_sensor, ws, exclude=None,
                       params=LOGODDS_DEFAULT, keep=None, stream=None):
    """params: (hit, miss, min, max, threshold) in the log-odds units."""
    g = make_grid(grid)
    n = pts.shape[0] if pts.dim() == 2 else pts.numel() // 3
    p = LogOdds(*[int(x) for x in params], 0)
    _check(lib().edt_update_logodds(ctypes.byref(g), _dev(logodds, torch.int16, "logodds", _n(g)),
                                    _dev(occ, torch.uint8, "occ", _n(g)),
                                    _dev(pts, torch.float32, "pts", 3 * n), n,
                                    _dev(T_map_sensor, torch.float32, "T_map_sensor", 12),
                                    _dev(keep, torch.uint8, "keep", n),
                                    _dev(exclude, torch.uint8, "exclude", _n(g)), ctypes.byref(p),
                                    _dev(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)),
           "edt_update_logodds")


OUTLIER_MAX_POINTS = 4194304


def edt_outlier_workspace_bytes(n_points: int) -> int:
    return int(lib().edt_outlier_workspace_bytes(int(n_points)))


def new_outlier_workspace(n_points: int, device="cuda"):
    return torch.empty(edt_outlier_workspace_bytes(n_points), dtype=torch.uint8, device=device)


def edt_outlier_filter(pts, keep, ws, k=8, radius=0.01, alpha=1.0, mean_dist=None, stats=None,
                       stream=None):
    """pts float32 [n, 3] (device); keep uint8 [n] out; mean_dist float32 [n]
    and stats float64 [3] (mu, sigma, threshold) optional outputs."""
    n = pts.shape[0]
    _check(lib().edt_outlier_filter(_dev(pts, torch.float32, "pts", 3 * n), n, int(k), float(radius),
                                    float(alpha), _dev(keep, torch.uint8, "keep", n),
                                    _dev(mean_dist, torch.float32, "mean_dist", n),
                                    _dev(stats, torch.float64, "stats", 3),
                                    _dev(ws, torch.uint8, "ws"), ws.numel(), _stream(stream)),
           "edt_outlier_filter")


def new_edt_cache(grid, device="cuda"):
    """A zeroed static-scene cache for edt_compute_cached."""
    n = int(lib().edt_cache_workspace_bytes(ctypes.byref(make_grid(grid))))
    return torch.zeros(n, dtype=torch.uint8, device=device)


def edt_cache_reset(grid, cache, stream=None):
    _check(lib().edt_cache_reset(ctypes.byref(make_grid(grid)), _dev(cache, torch.uint8, "cache"),
                                 cache.numel(), _stream(stream)), "edt_cache_reset")


def edt_compute_cached(grid, occ, d2, site, cache, stream=None):
    g = make_grid(grid)
    n = _n(g)
    _check(lib().edt_compute_cached(ctypes.byref(g), _dev(occ, torch.uint8, "occ", n),
                                    _dev(d2, torch.int32, "d2", n), _dev(site, torch.int32, "site", n),
                                    _dev(cache, torch.uint8, "cache"), cache.numel(), _stream(stream)),
           "edt_compute_cached")


def new_jfa_workspace(grid, device="cuda"):
    n = int(lib().edt_jfa_workspace_bytes(ctypes.byref(make_grid(grid))))
    return torch.empty(n, dtype=torch.uint8, device=device)


def edt_jfa(grid, occ, d2, site, ws, stream=None):
    """Jump flooding (approximate); outputs as edt_compute."""
    g = make_grid(grid)
    n = _n(g)
    _check(lib().edt_jfa(ctypes.byref(g), _dev(occ, torch.uint8, "occ", n), _dev(d2, torch.int32, "d2", n),
                         _dev(site, torch.int32, "site", n), _dev(ws, torch.uint8, "ws"), ws.numel(),
                         _stream(stream)), "edt_jfa")
