"""All-pairs reference EDT -- TEST INFRASTRUCTURE ONLY (pins the oracle).

The definition of the transform (Sec. III-C: the closest occupied voxel of
every voxel, i.e. the discrete Voronoi diagram of the occupied voxels) written
out directly: for every voxel, the minimum squared distance over every
occupied voxel, and the smallest linear index among the minimisers.
Quadratic in the voxel count, so only for small grids.
"""
from __future__ import annotations

import numpy as np

INT32_MAX = np.iinfo(np.int32).max


def coords(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], -1).astype(np.int64)


def brute_edt(occ: np.ndarray, tie: str = "min"):
    """(d2, site) by exhaustive search; tie = 'min' or 'max' linear index."""
    occ = np.asarray(occ)
    P = coords(occ.shape)
    S = np.flatnonzero(occ.ravel() != 0)
    n = P.shape[0]
    if S.size == 0:
        return (np.full(occ.shape, INT32_MAX, np.int32), np.full(occ.shape, -1, np.int32))
    d2 = np.empty(n, np.int64)
    site = np.empty(n, np.int64)
    chunk = max(1, (1 << 22) // S.size)
    Sc = P[S]
    for i0 in range(0, n, chunk):
        D = ((P[i0:i0 + chunk, None, :] - Sc[None, :, :]) ** 2).sum(-1)
        m = D.min(1)
        d2[i0:i0 + chunk] = m
        eq = D == m[:, None]
        if tie == "min":
            site[i0:i0 + chunk] = S[eq.argmax(1)]
        else:
            site[i0:i0 + chunk] = S[S.size - 1 - eq[:, ::-1].argmax(1)]
    return d2.reshape(occ.shape).astype(np.int32), site.reshape(occ.shape).astype(np.int32)
