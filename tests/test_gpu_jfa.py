"""Jump flooding on the GPU against the CPU oracle's jump flooding, bit for
bit (sites and d2), on ragged shapes, edge cases and the control-cycle map;
and the naive one-band-per-line tiling of the exact transform."""
import numpy as np
import pytest
import torch

import oracle
from paper_2407_02363_amd import edt, inputs
from tests.gpu_util import dev, gpu_edt, grid_of, say

pytestmark = pytest.mark.gpu


def gpu_jfa(occ):
    d = dev()
    g = grid_of(occ.shape)
    o = torch.from_numpy(np.ascontiguousarray(occ).ravel()).to(d)
    d2 = torch.full((occ.size,), -7, dtype=torch.int32, device=d)
    site = torch.full_like(d2, -7)
    edt.edt_jfa(g, o, d2, site, edt.new_jfa_workspace(g, d))
    torch.cuda.synchronize()
    return d2.cpu().numpy().reshape(occ.shape), site.cpu().numpy().reshape(occ.shape)


@pytest.mark.parametrize("shape,density", [((1, 1, 1), 1.0), ((1, 1, 1), 0.0), ((3, 5, 7), 0.1),
                                           ((33, 70, 65), 0.002), ((64, 64, 64), 0.01),
                                           ((6, 9, 700), 0.003), ((20, 31, 1), 0.05)])
def test_matches_oracle(shape, density):
    occ = inputs.random_grid(shape, density, sum(shape))
    say(f"[jfa] {shape} d={density}")
    d2, site = gpu_jfa(occ)
    rd2, rsite = oracle.jfa(occ)
    assert np.array_equal(d2, rd2) and np.array_equal(site, rsite)


def test_control_cycle_map():
    ci = inputs.cycle_inputs(0, n_frames=1)
    occ = np.zeros(ci.grid.shape, np.uint8)
    oracle.insert_points(ci.grid, occ, ci.frames[0], ci.T_map_cam)
    say("[jfa] 256x256x128 control-cycle map")
    d2, site = gpu_jfa(occ)
    rd2, rsite = oracle.jfa(occ)
    assert np.array_equal(d2, rd2) and np.array_equal(site, rsite)
    exact, _ = gpu_edt(occ)
    assert (d2 >= exact).all()
    say(f"[jfa] voxels off the exact transform: {np.mean(d2 != exact):.5f}")


def test_naive_tiling_is_exact():
    """One band per line in both passes (xy tile = xy group = 64, z tile = z
    group = 64): the paper's m1 = m2 = m3 = 1 baseline, same results."""
    occ = inputs.random_grid((70, 90, 130), 0.005, 4)
    d = dev()
    g = grid_of(occ.shape)
    o = torch.from_numpy(occ.ravel()).to(d)
    d2 = torch.empty(occ.size, dtype=torch.int32, device=d)
    site = torch.empty_like(d2)
    edt.edt_compute_tuned(g, o, d2, site, (64, 64, 64, 64))
    torch.cuda.synchronize()
    rd2, rsite = oracle.edt(occ)
    assert np.array_equal(d2.cpu().numpy().reshape(occ.shape), rd2)
    assert np.array_equal(site.cpu().numpy().reshape(occ.shape), rsite)
