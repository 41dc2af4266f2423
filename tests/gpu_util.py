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


def gpu_edt(occ: np.ndarray, grid=None):
    """(d2, site) from edt_compute on the GPU, as numpy arrays of occ's shape."""
    import torch
    from paper_2407_02363_amd import edt
    g = grid if grid is not None else grid_of(occ.shape)
    o = torch.from_numpy(np.ascontiguousarray(occ, np.uint8).ravel()).to(dev())
    n = occ.size
    d2 = torch.full((n,), -7, dtype=torch.int32, device=dev())
    site = torch.full((n,), -7, dtype=torch.int32, device=dev())
    edt.edt_compute(g, o, d2, site)
    torch.cuda.synchronize()
    return d2.cpu().numpy().reshape(occ.shape), site.cpu().numpy().reshape(occ.shape)
