"""Batched EDT (many maps of uneven size in one persistent launch) against
the CPU oracle map by map, every batch tiling, the batch autotuner, graph
replays of a batch, and argument errors."""
import numpy as np
import pytest
import torch

from paper_2407_02363_amd import edt, inputs
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu


def run_batch(occs, grids, tuning=None):
    d = dev()
    o = [torch.from_numpy(np.ascontiguousarray(x).ravel()).to(d) for x in occs]
    d2 = [torch.full((x.size,), -7, dtype=torch.int32, device=d) for x in occs]
    st = [torch.full((x.size,), -7, dtype=torch.int32, device=d) for x in occs]
    maps = edt.batch_maps(grids, o, d2, st)
    ws = edt.new_batch_workspace(len(grids), d)
    edt.edt_compute_batched(maps, ws, tuning)
    torch.cuda.synchronize()
    assert not edt.edt_batch_status(ws)
    return ([a.cpu().numpy().reshape(x.shape) for a, x in zip(d2, occs)],
            [a.cpu().numpy().reshape(x.shape) for a, x in zip(st, occs)], (o, d2, st, maps, ws))


def mixed_batch(seed):
    r = inputs.rng(seed)
    shapes = [(1, 1, 1), (3, 5, 7), (17, 64, 64), (40, 70, 130), (64, 128, 128), (128, 97, 65),
              (9, 256, 31), (100, 100, 100), (33, 33, 33), (5, 200, 192)]
    occs = []
    for i, sh in enumerate(shapes):
        dens = [0.0, 0.3, 0.01, 0.002, 0.05, 0.0005, 0.02, 0.001, 1.0, 0.01][i]
        occs.append(inputs.random_grid(sh, dens, seed * 100 + i))
    occs[7] = inputs.single_site_grid((100, 100, 100), (3, 97, 50))
    grids = [inputs.Grid(sh[2], sh[1], sh[0]) for sh in shapes]
    return occs, grids


def check(occs, d2s, sites, oracle_lib, tag):
    for i, occ in enumerate(occs):
        rd2, rsite = oracle_lib.edt(occ)
        assert np.array_equal(d2s[i], rd2), f"{tag}: map {i} {occ.shape} d2"
        assert np.array_equal(sites[i], rsite), f"{tag}: map {i} {occ.shape} site"


def test_mixed_batch_matches_oracle(oracle_lib):
    occs, grids = mixed_batch(1)
    say(f"[batch] mixed {len(occs)} maps")
    d2s, sites, _ = run_batch(occs, grids)
    check(occs, d2s, sites, oracle_lib, "mixed")


def lean_batch(seed):
    """Maps the lean batch kernel takes: rows of 64-512 voxels, up to 256 rows
    and 128 slices, ragged, sparse to dense, one empty."""
    shapes = [(128, 256, 256), (64, 64, 64), (97, 130, 65), (1, 40, 64), (128, 255, 200), (33, 1, 300),
              (70, 200, 512), (5, 256, 64)]
    dens = [0.001, 0.3, 0.01, 0.05, 0.0005, 0.02, 0.0, 0.002]
    occs = [inputs.random_grid(sh, d, seed * 50 + i) for i, (sh, d) in enumerate(zip(shapes, dens))]
    occs[0][3, 200, 17] = 1
    grids = [inputs.Grid(sh[2], sh[1], sh[0]) for sh in shapes]
    return occs, grids


def test_lean_batch_kernel(oracle_lib):
    """The persistent batch kernel with the lean tiles (records, xy, then z
    tiles two per work-group, each phase waiting for the map's previous one):
    every map against the oracle, by default and asked for as tiles (64, 64),
    twice in a row on one workspace; asking for it on a batch it cannot take
    is an error."""
    occs, grids = lean_batch(1)
    say(f"[batch] lean kernel, {len(occs)} maps")
    for tiles in (None, (64, 64)):
        d2s, sites, keep = run_batch(occs, grids, tiles)
        check(occs, d2s, sites, oracle_lib, f"lean {tiles}")
        o, d2, st, maps, ws = keep
        for a in d2 + st:
            a.fill_(-7)
        edt.edt_compute_batched(maps, ws, tiles)
        torch.cuda.synchronize()
        assert not edt.edt_batch_status(ws)
        check(occs, [a.cpu().numpy().reshape(x.shape) for a, x in zip(d2, occs)],
              [a.cpu().numpy().reshape(x.shape) for a, x in zip(st, occs)], oracle_lib, f"lean again {tiles}")
    mocc, mgrids = mixed_batch(5)
    with pytest.raises(edt.EdtError):
        run_batch(mocc, mgrids, (64, 64))


@pytest.mark.parametrize("tiles", [(16, 16), (16, 32), (16, 64), (32, 16), (32, 32), (32, 64)])
def test_every_batch_tiling(oracle_lib, tiles):
    occs, grids = mixed_batch(2)
    say(f"[batch] tiles {tiles}")
    d2s, sites, _ = run_batch(occs, grids, tiles)
    check(occs, d2s, sites, oracle_lib, f"tiles {tiles}")


def test_batched_cycle_maps(oracle_lib):
    """Uneven maps filled from their own depth frames (the batched workload)."""
    bi = inputs.batch_inputs(seed=3, n_maps=6, n_states=2, min_points=20_000, max_points=60_000)
    occs = []
    for g, pts, T in zip(bi.grids, bi.clouds, bi.T_map_cam):
        occ = np.zeros(g.shape, np.uint8)
        oracle_lib.insert_points(g, occ, pts, T)
        occs.append(occ)
    say(f"[batch] cycle maps {[g.shape for g in bi.grids]}")
    d2s, sites, _ = run_batch(occs, bi.grids)
    check(occs, d2s, sites, oracle_lib, "cycle maps")


def test_batch_autotune(oracle_lib):
    occs, grids = mixed_batch(4)
    d = dev()
    o = [torch.from_numpy(x.ravel()).to(d) for x in occs]
    d2 = [torch.empty(x.size, dtype=torch.int32, device=d) for x in occs]
    st = [torch.empty(x.size, dtype=torch.int32, device=d) for x in occs]
    maps = edt.batch_maps(grids, o, d2, st)
    ws = edt.new_batch_workspace(len(grids), d)
    tiles, us = edt.edt_autotune_batched(maps, ws, reps=2)
    say(f"[batch] autotune -> {tiles} {us:.1f} us")
    check(occs, [a.cpu().numpy().reshape(x.shape) for a, x in zip(d2, occs)],
          [a.cpu().numpy().reshape(x.shape) for a, x in zip(st, occs)], oracle_lib, "autotuned")


def test_batch_graph_replays(oracle_lib):
    occs, grids = mixed_batch(5)
    d2s, sites, (o, d2, st, maps, ws) = run_batch(occs, grids)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        edt.edt_compute_batched(maps, ws)
    for rep in range(3):
        for a in d2 + st:
            a.fill_(-7)
        torch.cuda.synchronize()
        say(f"[batch] graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        got_d2 = [a.cpu().numpy().reshape(x.shape) for a, x in zip(d2, occs)]
        got_st = [a.cpu().numpy().reshape(x.shape) for a, x in zip(st, occs)]
        for i in range(len(occs)):
            assert np.array_equal(got_d2[i], d2s[i]) and np.array_equal(got_st[i], sites[i])
        # eager work between replays
        edt.edt_compute(grids[4], o[4], d2[4], st[4])
        torch.cuda.synchronize()


def test_batch_errors():
    d = dev()
    ws = edt.new_batch_workspace(2, d)
    o = torch.zeros(8, dtype=torch.uint8, device=d)
    a = torch.zeros(8, dtype=torch.int32, device=d)
    g = inputs.Grid(2, 2, 2)
    maps = edt.batch_maps([g], [o], [a], [a.clone()])
    with pytest.raises(edt.EdtError) as e:
        edt.edt_compute_batched(maps, ws[:4])
    assert e.value.status == -3
    big = inputs.Grid(600, 1, 1)
    o2 = torch.zeros(600, dtype=torch.uint8, device=d)
    b = torch.zeros(600, dtype=torch.int32, device=d)
    with pytest.raises(edt.EdtError) as e:
        edt.edt_compute_batched(edt.batch_maps([big], [o2], [b], [b.clone()]), ws)
    assert e.value.status == -5
    with pytest.raises(edt.EdtError) as e:
        edt.edt_compute_batched(maps, ws, (64, 64))
    assert e.value.status == -5


def test_batch_cycle_plain_batched_graph(oracle_lib):
    """The batched cycle: per-map launches, one persistent launch, and the
    graph-captured batched cycle give the same bytes as the oracle."""
    from paper_2407_02363_amd.batch_cycle import BatchCycle
    bi = inputs.batch_inputs(seed=6, n_maps=5, n_states=3, min_points=10_000, max_points=40_000)
    bc = BatchCycle(bi)
    refs = []
    for i, g in enumerate(bi.grids):
        occ = np.zeros(g.shape, np.uint8)
        oracle_lib.insert_points(g, occ, bi.clouds[i], bi.T_map_cam[i])
        d2, site = oracle_lib.edt(occ)
        c = bi.centres[i].reshape(-1, 3)
        r = np.tile(bi.sphere_radii[i], bi.centres[i].shape[0])
        refs.append((d2, site, oracle_lib.query_spheres(g, d2, site, c, r)))

    def verify(tag):
        torch.cuda.synchronize()
        for i, g in enumerate(bi.grids):
            assert np.array_equal(bc.d2[i].cpu().numpy().reshape(g.shape), refs[i][0]), (tag, i)
            assert np.array_equal(bc.site[i].cpu().numpy().reshape(g.shape), refs[i][1]), (tag, i)
            assert np.array_equal(bc.out[i].cpu().numpy().view(np.uint32), refs[i][2]), (tag, i)

    say("[batch cycle] plain")
    bc.run_plain()
    verify("plain")
    say("[batch cycle] batched")
    bc.run_batched()
    verify("batched")
    say("[batch cycle] many")
    for t in bc.d2 + bc.site:
        t.fill_(-7)
    bc.run_many()
    verify("many")
    graph_many = bc.capture(bc.run_many)
    for t in bc.d2 + bc.site:
        t.fill_(-7)
    graph_many.replay()
    verify("many graph")
    graph = bc.capture(bc.run_batched)
    for rep in range(3):
        for t in bc.d2 + bc.site:
            t.fill_(-7)
        say(f"[batch cycle] graph replay {rep}")
        graph.replay()
        verify(f"graph {rep}")
        bc.run_plain()
        torch.cuda.synchronize()


def run_many(occs, grids, tuning=None):
    d = dev()
    o = [torch.from_numpy(np.ascontiguousarray(x).ravel()).to(d) for x in occs]
    d2 = [torch.full((x.size,), -7, dtype=torch.int32, device=d) for x in occs]
    st = [torch.full((x.size,), -7, dtype=torch.int32, device=d) for x in occs]
    maps = edt.batch_maps(grids, o, d2, st)
    edt.edt_compute_many(maps, tuning)
    torch.cuda.synchronize()
    return ([a.cpu().numpy().reshape(x.shape) for a, x in zip(d2, occs)],
            [a.cpu().numpy().reshape(x.shape) for a, x in zip(st, occs)])


@pytest.mark.parametrize("tiles", [None, (16, 8, 256), (32, 32, 128), (64, 16, 64), (32, 64, 256)])
def test_many_matches_oracle(oracle_lib, tiles):
    """One launch per pass over maps of different shapes (a map with an axis
    above 512 takes every map onto the 64-bit envelope test)."""
    occs, grids = mixed_batch(3)
    if tiles is None:
        occs.append(inputs.random_grid((6, 9, 700), 0.01, 77))
        grids.append(inputs.Grid(700, 9, 6))
    say(f"[many] {len(occs)} maps tiles {tiles}")
    d2s, sites = run_many(occs, grids, tiles)
    check(occs, d2s, sites, oracle_lib, f"many {tiles}")


def test_many_48_maps_of_one_shape(oracle_lib):
    """48 maps of one shape (the self-map labeler's case), every map against
    the oracle."""
    sh = (24, 40, 36)
    occs = [inputs.random_grid(sh, 0.003 * (1 + i % 5), 500 + i) for i in range(edt.BATCH_MAX)]
    grids = [inputs.Grid(sh[2], sh[1], sh[0])] * len(occs)
    d2s, sites = run_many(occs, grids)
    check(occs, d2s, sites, oracle_lib, "48 maps")


def test_batch_cycle_configured_size(oracle_lib):
    """The batched workload at its configured size: 32 maps with axes uniform
    in 64..256 x 64..256 x 64..128, each with its own frame of 50k-300k
    points and 16 look-ahead states x 20 spheres.  Every map's d2, site and
    query records against the oracle, for the persistent launch, one launch
    per pass, and both captured as graphs."""
    from paper_2407_02363_amd.batch_cycle import BatchCycle
    bi = inputs.batch_inputs(seed=0, n_maps=32)
    say(f"[batch cycle 32] {sum(g.n for g in bi.grids)} voxels, "
        f"{sum(c.shape[0] for c in bi.clouds)} points")
    bc = BatchCycle(bi)
    refs = []
    for i, g in enumerate(bi.grids):
        occ = np.zeros(g.shape, np.uint8)
        oracle_lib.insert_points(g, occ, bi.clouds[i], bi.T_map_cam[i])
        d2, site = oracle_lib.edt(occ)
        c = bi.centres[i].reshape(-1, 3)
        r = np.tile(bi.sphere_radii[i], bi.centres[i].shape[0])
        refs.append((d2, site, oracle_lib.query_spheres(g, d2, site, c, r)))

    def verify(tag):
        torch.cuda.synchronize()
        for i, g in enumerate(bi.grids):
            assert np.array_equal(bc.d2[i].cpu().numpy().reshape(g.shape), refs[i][0]), (tag, i)
            assert np.array_equal(bc.site[i].cpu().numpy().reshape(g.shape), refs[i][1]), (tag, i)
            assert np.array_equal(bc.out[i].cpu().numpy().view(np.uint32), refs[i][2]), (tag, i)

    def poison():
        for t in bc.d2 + bc.site:
            t.fill_(-7)

    for name, fn in (("batched", bc.run_batched), ("many", bc.run_many)):
        say(f"[batch cycle 32] {name}")
        poison()
        fn()
        verify(name)
        assert not edt.edt_batch_status(bc.ws)
        graph = bc.capture(fn)
        for rep in range(2):
            poison()
            torch.cuda.synchronize()
            say(f"[batch cycle 32] {name} graph replay {rep}")
            graph.replay()
            verify(f"{name} graph {rep}")
        del graph
    assert not edt.edt_batch_status(bc.ws)


def gated_case(case):
    """Maps that take each path of the two passes: lean xy + lean z, plain xy,
    row records + xy from records, the 64-bit (wide) envelope test, and
    explicit tiles."""
    tuning = None
    if case == "lean":
        shapes = [(128, 128, 128), (100, 200, 64), (64, 256, 96), (128, 128, 128), (77, 64, 64)]
        occs = [inputs.random_grid(sh, 0.002 * (i + 1), 900 + i) for i, sh in enumerate(shapes)]
        grids = [inputs.Grid(sh[2], sh[1], sh[0]) for sh in shapes]
    elif case == "rows":
        shapes = [(16, 300, 256), (8, 260, 300), (24, 280, 260)]
        occs = [inputs.random_grid(sh, 0.001 * (i + 1), 920 + i) for i, sh in enumerate(shapes)]
        grids = [inputs.Grid(sh[2], sh[1], sh[0]) for sh in shapes]
    else:
        occs, grids = mixed_batch(4)
        if case == "wide":
            occs, grids = occs[:5], grids[:5]
            occs.append(inputs.random_grid((6, 9, 700), 0.01, 78))
            grids.append(inputs.Grid(700, 9, 6))
        elif case == "tiles":
            tuning = (32, 32, 128)
    return occs, grids, tuning


@pytest.mark.parametrize("case", ["lean", "rows", "mixed", "wide", "tiles"])
def test_many_gated(oracle_lib, case):
    """edt_compute_many_gated: a map whose device gate is 0 keeps its d2 and
    site bit for bit, every other map matches the oracle; flipping the gates
    in place transforms the rest; a captured graph reads the gates anew on
    every replay."""
    occs, grids, tuning = gated_case(case)
    d = dev()
    n = len(occs)
    say(f"[many gated] {case}: {n} maps, tiles {tuning}")
    refs = [oracle_lib.edt(o) for o in occs]
    o = [torch.from_numpy(np.ascontiguousarray(x).ravel()).to(d) for x in occs]
    d2 = [torch.empty(x.size, dtype=torch.int32, device=d) for x in occs]
    st = [torch.empty(x.size, dtype=torch.int32, device=d) for x in occs]
    maps = edt.batch_maps(grids, o, d2, st)
    gates = torch.from_numpy((np.arange(n) % 2).astype(np.int32)).to(d)

    def poison():
        for i in range(n):
            d2[i].fill_(-7 - i)
            st[i].fill_(-100 - i)

    def verify(on, tag):
        torch.cuda.synchronize()
        for i, x in enumerate(occs):
            a = d2[i].cpu().numpy().reshape(x.shape)
            b = st[i].cpu().numpy().reshape(x.shape)
            if on[i]:
                assert np.array_equal(a, refs[i][0]) and np.array_equal(b, refs[i][1]), (tag, i)
            else:
                assert (a == -7 - i).all() and (b == -100 - i).all(), (tag, i, "touched")

    poison()
    edt.edt_compute_many_gated(maps, gates, tuning)
    on = [bool(i % 2) for i in range(n)]
    verify(on, "first")
    gates.copy_(1 - gates)
    edt.edt_compute_many_gated(maps, gates, tuning)
    verify([True] * n, "flipped")
    if case != "lean":
        return
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, capture_error_mode="thread_local"):
        edt.edt_compute_many_gated(maps, gates, tuning)
    torch.cuda.synchronize()
    for rep, pattern in enumerate(([1, 0, 0, 1, 1], [0, 1, 1, 0, 0], [0, 0, 0, 0, 0], [1, 1, 1, 1, 1])):
        poison()
        gates.copy_(torch.tensor(pattern, dtype=torch.int32))
        torch.cuda.synchronize()
        say(f"[many gated] graph replay {rep} gates {pattern}")
        graph.replay()
        verify([bool(p) for p in pattern], f"graph {rep}")
