"""Helpers for the GPU parity tests: run the HIP path through the C-ABI."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev():
    import torch
    return torch.device("cuda:0")


def grid_of(shape, origin=(0.0, 0.0, 0.0), voxel=0.01):
    from paper_2407_02363_amd import inputs
    nz, ny, nx = shape
    return inputs.Grid(nx, ny, nz, origin, voxel)


def gpu_edt(occ: np.ndarray, grid=None, occ_offset: int = 0):
    """(d2, site) from edt_compute on the GPU, as numpy arrays of occ's shape.
    occ_offset > 0 places the occupancy bytes that far into a larger device
    buffer, so the pointer handed over is not 16-byte aligned."""
    import torch
    from paper_2407_02363_amd import edt
    g = grid if grid is not None else grid_of(occ.shape)
    n = occ.size
    flat = torch.from_numpy(np.ascontiguousarray(occ, np.uint8).ravel())
    if occ_offset:
        buf = torch.full((n + occ_offset + 16,), 0xFF, dtype=torch.uint8, device=dev())
        o = buf[occ_offset:occ_offset + n]
        o.copy_(flat.to(dev()))
    else:
        o = flat.to(dev())
    d2 = torch.full((n,), -7, dtype=torch.int32, device=dev())
    site = torch.full((n,), -7, dtype=torch.int32, device=dev())
    edt.edt_compute(g, o, d2, site)
    torch.cuda.synchronize()
    return d2.cpu().numpy().reshape(occ.shape), site.cpu().numpy().reshape(occ.shape)
