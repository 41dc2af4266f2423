"""The allocation-free batched entry point (edt_compute_batched_noalloc)
against edt_compute_batched with a caller's workspace: bit-exact d2 and site
on two calls in a row, the second with a smaller batch of smaller maps, and
the timed-out flag clear.  Calls through the C-ABI."""
import numpy as np
import pytest
import torch

from paper_2407_02363_amd import edt, inputs
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu


def batch(shapes, seed):
    occs = [inputs.random_grid(sh, [0.002, 0.03, 0.0005, 0.2][i % 4], seed * 10 + i)
            for i, sh in enumerate(shapes)]
    grids = [inputs.Grid(sh[2], sh[1], sh[0]) for sh in shapes]
    return occs, grids


def outputs(occs):
    d = dev()
    o = [torch.from_numpy(np.ascontiguousarray(x).ravel()).to(d) for x in occs]
    d2 = [torch.full((x.size,), -7, dtype=torch.int32, device=d) for x in occs]
    st = [torch.full((x.size,), -7, dtype=torch.int32, device=d) for x in occs]
    return o, d2, st


def test_noalloc_matches_workspace_call(oracle_lib):
    calls = [([(64, 128, 128), (100, 64, 200), (33, 70, 65), (128, 96, 96), (17, 20, 300), (50, 50, 50)], 1),
             ([(40, 64, 64), (9, 30, 70), (20, 20, 20)], 2)]
    flag = torch.full((1,), -1, dtype=torch.int32, device=dev())
    for shapes, seed in calls:
        occs, grids = batch(shapes, seed)
        say(f"[noalloc] {len(shapes)} maps {shapes}")
        o, d2a, sta = outputs(occs)
        ws = edt.new_batch_workspace(len(grids), dev())
        edt.edt_compute_batched(edt.batch_maps(grids, o, d2a, sta), ws)
        _, d2b, stb = outputs(occs)
        flag.fill_(-1)
        maps_b = edt.batch_maps(grids, o, d2b, stb)
        edt.edt_compute_batched_noalloc(maps_b, timed_out=flag)
        torch.cuda.synchronize()
        assert not edt.edt_batch_status(ws)
        assert int(flag.item()) == 0
        for i, occ in enumerate(occs):
            assert torch.equal(d2a[i], d2b[i]), f"map {i} d2"
            assert torch.equal(sta[i], stb[i]), f"map {i} site"
            rd2, rsite = oracle_lib.edt(occ)
            assert np.array_equal(d2b[i].cpu().numpy().reshape(occ.shape), rd2), f"map {i} d2 vs oracle"
            assert np.array_equal(stb[i].cpu().numpy().reshape(occ.shape), rsite), f"map {i} site vs oracle"


def test_noalloc_rejects_too_many_maps():
    grids = [inputs.Grid(4, 4, 4)] * (edt.BATCH_MAX + 1)
    t = [torch.zeros(64, dtype=torch.uint8, device=dev()) for _ in grids]
    d = [torch.zeros(64, dtype=torch.int32, device=dev()) for _ in grids]
    maps = edt.batch_maps(grids, t, d, d)
    with pytest.raises(edt.EdtError) as e:
        edt.edt_compute_batched_noalloc(maps)
    assert e.value.status == -1
