"""GPU parity of edt_compute against the CPU oracle: bit-exact int32 d2 and
nearest-site index, on the seeded workloads and on edge cases (empty, full,
single site, degenerate lines, ragged dims that leave partial tiles, dims
that select every tile width and the 64-bit envelope path)."""
import numpy as np
import pytest

from paper_2407_02363_amd import inputs
from tests.gpu_util import gpu_edt, say

pytestmark = pytest.mark.gpu


def assert_same(occ, oracle_lib, tag):
    say(f"[edt parity] {tag} shape={occ.shape}")
    d2, site = gpu_edt(occ)
    rd2, rsite = oracle_lib.edt(occ)
    bad_d = int((d2 != rd2).sum())
    bad_s = int((site != rsite).sum())
    assert bad_d == 0 and bad_s == 0, f"{tag}: {bad_d} d2 and {bad_s} site mismatches"


def assert_same_many(occ, oracle_lib, tag, min_tiles=1100):
    """occ as enough separate maps of one edt_compute_many launch that the
    launch has more than min_tiles xy tiles of 64 columns (past what two
    work-groups per CU hold, where the xy tiles of maps up to 256 columns
    switch to 16-bit stack entries); every copy against the oracle."""
    import torch
    from paper_2407_02363_amd import edt
    from tests.gpu_util import dev, grid_of
    nz, ny, nx = occ.shape
    k = min(edt.BATCH_MAX, min_tiles // (nz * ((nx + 63) // 64)) + 1)
    say(f"[edt parity] {tag} shape={occ.shape} as {k} maps of one launch")
    g = grid_of(occ.shape)
    flat = torch.from_numpy(np.ascontiguousarray(occ, np.uint8).ravel()).to(dev())
    occs = [flat.clone() for _ in range(k)]
    d2s = [torch.full((occ.size,), -7, dtype=torch.int32, device=dev()) for _ in range(k)]
    sites = [torch.full((occ.size,), -7, dtype=torch.int32, device=dev()) for _ in range(k)]
    edt.edt_compute_many(edt.batch_maps([g] * k, occs, d2s, sites))
    torch.cuda.synchronize()
    rd2, rsite = oracle_lib.edt(occ)
    for i in range(k):
        bad_d = int((d2s[i].cpu().numpy().reshape(occ.shape) != rd2).sum())
        bad_s = int((sites[i].cpu().numpy().reshape(occ.shape) != rsite).sum())
        assert bad_d == 0 and bad_s == 0, f"{tag} copy {i}: {bad_d} d2 and {bad_s} site mismatches"


@pytest.mark.parametrize("seed", range(4))
def test_boxes_64cubed(oracle_lib, seed):
    assert_same(inputs.boxes_grid(64, seed=seed), oracle_lib, f"boxes64 seed{seed}")


@pytest.mark.parametrize("density", [0.001, 0.02, 0.3, 0.7])
def test_random_16cubed_and_brute(oracle_lib, density):
    from oracle.brute import brute_edt
    occ = inputs.random_grid((16, 16, 16), density, 3)
    d2, site = gpu_edt(occ)
    bd, bs = brute_edt(occ)
    assert np.array_equal(d2, bd) and np.array_equal(site, bs)


SHAPES = [
    (1, 1, 1), (1, 1, 17), (1, 17, 1), (17, 1, 1), (3, 5, 7), (2, 1, 130),
    (65, 63, 70),        # ragged tiles in x, odd band lengths
    (40, 257, 100),      # ny > 256: 32-wide xy tiles
    (129, 30, 66),       # nz > 128: 32-wide z tiles
    (300, 20, 129),      # nz > 256: 16-wide z tiles
    (20, 520, 33),       # ny > 512: 16-wide xy tiles, 64-bit envelope test
    (700, 9, 11),        # nz > 512: 8-wide z tiles, 64-bit envelope test
    (7, 6, 1000),        # nx > 512: many words per row, 64-bit envelope test
    (6, 40, 301),        # row records read byte by byte (nx >= 256, not a multiple of 4)
    (5, 33, 300),        # row records read 4 bytes per lane, last 256-byte chunk partial
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("density", [0.0005, 0.05])
def test_random_shapes(oracle_lib, shape, density):
    occ = inputs.random_grid(shape, density, sum(shape))
    assert_same(occ, oracle_lib, f"random d={density}")


@pytest.mark.parametrize("shape,offset", [((5, 64, 128), 1), ((9, 33, 70), 7), ((4, 20, 256), 15),
                                          ((2, 3, 5), 3), ((1, 1, 1), 9), ((6, 17, 1000), 5)])
def test_unaligned_occ_and_byte_values(oracle_lib, shape, offset):
    """occ not 16-byte aligned, bytes around it set to 0xFF (they must not be
    read as map voxels), and occupied voxels holding arbitrary nonzero byte
    values (any nonzero byte is occupied)."""
    g = np.random.Generator(np.random.PCG64(offset))
    occ = inputs.random_grid(shape, 0.02, offset)
    occ = (occ * g.integers(1, 256, size=occ.shape)).astype(np.uint8)
    say(f"[edt parity] unaligned offset={offset} shape={shape}")
    d2, site = gpu_edt(occ, occ_offset=offset)
    rd2, rsite = oracle_lib.edt(occ)
    assert np.array_equal(d2, rd2) and np.array_equal(site, rsite)


def test_empty_full_single(oracle_lib):
    assert_same(np.zeros((33, 70, 65), np.uint8), oracle_lib, "empty")
    assert_same(np.ones((9, 70, 65), np.uint8), oracle_lib, "full")
    for s in [(0, 0, 0), (64, 69, 32), (17, 3, 20)]:
        assert_same(inputs.single_site_grid((33, 70, 65), s), oracle_lib, f"single {s}")


def test_extreme_axes_1024(oracle_lib):
    """Longest axes the API allows (keys up to ~1023^2): a site at each end of
    a 1024-long line, and a lone site at the far end."""
    for shape, s in [((1, 1, 1024), (1023, 0, 0)), ((1, 1024, 2), (1, 1023, 0)),
                     ((1024, 1, 3), (2, 0, 1023))]:
        occ = inputs.single_site_grid(shape, s)
        assert_same(occ, oracle_lib, f"lone site {shape}")
        occ.reshape(-1)[0] = 1
        assert_same(occ, oracle_lib, f"two ends {shape}")


def test_two_far_corners_wide(oracle_lib):
    """Two sites at opposite corners of a 600 x 600 x 8 map: large keys and
    position gaps on every axis (64-bit envelope test)."""
    occ = np.zeros((8, 600, 600), np.uint8)
    occ[0, 0, 0] = 1
    occ[7, 599, 599] = 1
    occ[3, 599, 0] = 1
    assert_same(occ, oracle_lib, "far corners")


def test_control_cycle_map(oracle_lib):
    """256 x 256 x 128 map from the synthetic depth camera (1 cm voxels)."""
    ci = inputs.cycle_inputs(0, n_frames=1)
    occ = np.zeros(ci.grid.shape, np.uint8)
    oracle_lib.insert_points(ci.grid, occ, ci.frames[0], ci.T_map_cam)
    assert_same(occ, oracle_lib, "cycle map")


def test_large_blobs_512(oracle_lib):
    """512^3 at 5% clustered-blob occupancy, the large-map workload."""
    occ = inputs.blobs_grid(512)
    assert_same(occ, oracle_lib, "blobs512")


def test_deterministic(oracle_lib):
    occ = inputs.boxes_grid(64, seed=9)
    a = gpu_edt(occ)
    b = gpu_edt(occ)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("shape", [(128, 256, 256), (37, 90, 130), (64, 64, 64)])
def test_every_tiling_is_identical(oracle_lib, shape):
    """Tile widths (band counts) change the launch, never the result."""
    import torch
    from paper_2407_02363_amd import edt
    from tests.gpu_util import dev, grid_of
    occ = inputs.random_grid(shape, 0.003, 17)
    occ[shape[0] // 2, :, 5] = 1
    rd2, rsite = oracle_lib.edt(occ)
    g = grid_of(shape)
    o = torch.from_numpy(occ.ravel()).to(dev())
    d2 = torch.empty(occ.size, dtype=torch.int32, device=dev())
    site = torch.empty_like(d2)
    combos = [(xt, zt, 256, 256) for xt in (16, 32, 64) for zt in (8, 16, 32, 64)]
    combos += [(32, zt, zg, 256) for zg in (64, 128) for zt in (8, 16, 32, 64) if zt <= zg]
    combos += [(xt, 16, 256, xg) for xg in (64, 128) for xt in (16, 32, 64) if xt <= xg]
    combos += [(64, 64, 64, 64)]   # one band per line in both passes (the naive variant)
    combos += [(xt, 64, 256, 512) for xt in (32, 64)]   # 512-thread xy work-groups
    combos += [(32, 64, 512, 256)]                       # 512-thread z work-groups
    for xt, zt, zg, xg in combos:
        if True:
            say(f"[tiling] {shape} xy={xt}/{xg} z={zt}/{zg}")
            d2.fill_(-7)
            site.fill_(-7)
            try:
                edt.edt_compute_tuned(g, o, d2, site, (xt, zt, zg, xg))
            except edt.EdtError as e:
                assert e.status == -5   # tile needs more LDS than the device has
                continue
            torch.cuda.synchronize()
            assert np.array_equal(d2.cpu().numpy().reshape(shape), rd2), (xt, zt, zg, xg)
            assert np.array_equal(site.cpu().numpy().reshape(shape), rsite), (xt, zt, zg, xg)


@pytest.mark.parametrize("seed,gap", [(0, False), (1, False), (2, True)])
def test_sparse_slices_every_band_layout(oracle_lib, seed, gap):
    """Most slices empty, the rest holding one to three voxels far apart:
    along z every column sees few sites with very uneven heights, so bands
    are often empty or hold a single site and merges pop across several
    bands (with gap, only the first and last 24 slices hold voxels, so the
    middle bands are empty).  Every z tiling (1 to 8 bands per column) and
    both xy group sizes must match the oracle."""
    import torch
    from paper_2407_02363_amd import edt
    from tests.gpu_util import dev, grid_of
    shape = (128, 40, 96)
    g = inputs.rng(100 + seed)
    occ = np.zeros(shape, np.uint8)
    for z in range(shape[0]):
        if gap and 24 <= z < shape[0] - 24:
            continue
        if g.uniform() < (0.3 if gap else 0.12):
            for _ in range(int(g.integers(1, 4))):
                occ[z, g.integers(0, shape[1]), g.integers(0, shape[2])] = 1
    rd2, rsite = oracle_lib.edt(occ)
    grid = grid_of(shape)
    o = torch.from_numpy(occ.ravel()).to(dev())
    d2 = torch.empty(occ.size, dtype=torch.int32, device=dev())
    site = torch.empty_like(d2)
    combos = [(32, zt, zg, 256) for zg in (64, 128, 256) for zt in (8, 16, 32, 64) if zt <= zg]
    combos += [(32, 64, 512, 256), (32, 64, 256, 512), (64, 64, 256, 512)]
    for xt, zt, zg, xg in combos:
        say(f"[sparse slices] seed {seed} gap {gap} xy={xt}/{xg} z={zt}/{zg}")
        d2.fill_(-7)
        site.fill_(-7)
        edt.edt_compute_tuned(grid, o, d2, site, (xt, zt, zg, xg))
        torch.cuda.synchronize()
        assert np.array_equal(d2.cpu().numpy().reshape(shape), rd2), (xt, zt, zg, xg)
        assert np.array_equal(site.cpu().numpy().reshape(shape), rsite), (xt, zt, zg, xg)


def test_autotune_keeps_results(oracle_lib):
    import torch
    from paper_2407_02363_amd import edt
    from tests.gpu_util import dev, grid_of
    occ = inputs.boxes_grid(64, seed=3)
    g = grid_of(occ.shape)
    o = torch.from_numpy(occ.ravel()).to(dev())
    d2 = torch.empty(occ.size, dtype=torch.int32, device=dev())
    site = torch.empty_like(d2)
    tiles, us = edt.edt_autotune(g, o, d2, site, reps=3)
    say(f"[autotune] 64^3 -> {tiles} {us:.1f} us")
    assert us > 0 and edt.edt_default_tuning(g) == tiles
    rd2, rsite = oracle_lib.edt(occ)
    assert np.array_equal(d2.cpu().numpy().reshape(occ.shape), rd2)
    d2.fill_(0)
    edt.edt_compute(g, o, d2, site)
    torch.cuda.synchronize()
    assert np.array_equal(d2.cpu().numpy().reshape(occ.shape), rd2)
    assert np.array_equal(site.cpu().numpy().reshape(occ.shape), rsite)


def test_autotuned_tiles_survive_a_saved_cache(oracle_lib, tmp_path):
    """The autotuner's choice goes into the cache under this device's
    architecture, a saved cache restores it after the cache is cleared (the
    heuristic tiles apply in between), and the transform with the restored
    tiles is exact."""
    import torch
    from paper_2407_02363_amd import edt
    from tests.gpu_util import dev, grid_of
    occ = inputs.boxes_grid(48, seed=4)
    g = grid_of(occ.shape)
    o = torch.from_numpy(occ.ravel()).to(dev())
    d2 = torch.empty(occ.size, dtype=torch.int32, device=dev())
    site = torch.empty_like(d2)
    edt.edt_tuning_cache_clear()
    heuristic = edt.edt_default_tuning(g)
    tiles, _ = edt.edt_autotune(g, o, d2, site, reps=2)
    path = tmp_path / "tiles.txt"
    assert edt.edt_tuning_cache_save(path) == 1
    line = path.read_text().splitlines()[1].split()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    assert line[:5] == ["single", arch, "48", "48", "48"], line
    assert (int(line[6]), int(line[9]), int(line[10]), int(line[7])) == tiles
    edt.edt_tuning_cache_clear()
    assert edt.edt_default_tuning(g) == heuristic
    assert edt.edt_tuning_cache_load(path) == 1
    assert edt.edt_default_tuning(g) == tiles
    d2.fill_(-1)
    edt.edt_compute(g, o, d2, site)
    torch.cuda.synchronize()
    rd2, rsite = oracle_lib.edt(occ)
    assert np.array_equal(d2.cpu().numpy().reshape(occ.shape), rd2)
    assert np.array_equal(site.cpu().numpy().reshape(occ.shape), rsite)
    edt.edt_tuning_cache_clear()


def test_cached_transform_skips_only_unchanged_maps(oracle_lib):
    """edt_compute_cached: the first call and every call after a change give
    the oracle's result; a call on an unchanged map (occupied / free
    unchanged, whatever the nonzero byte values) leaves d2 and site as they
    are; the same holds through graph replays."""
    import torch
    from paper_2407_02363_amd import edt
    from tests.gpu_util import dev
    d = dev()
    shape = (40, 70, 65)
    g = inputs.Grid(shape[2], shape[1], shape[0])
    occ_np = inputs.random_grid(shape, 0.01, 3)
    buf = torch.zeros(occ_np.size + 3, dtype=torch.uint8, device=d)
    for off in (0, 3):                          # aligned and unaligned occ
        say(f"[cached] offset {off}")
        o = buf[off:off + occ_np.size]
        o.copy_(torch.from_numpy(occ_np.ravel()))
        d2 = torch.full((occ_np.size,), -7, dtype=torch.int32, device=d)
        site = torch.full_like(d2, -7)
        cache = edt.new_edt_cache(g, d)
        rd2, rs = oracle_lib.edt(occ_np)

        def check(ref_d2, ref_s):
            torch.cuda.synchronize()
            assert np.array_equal(d2.cpu().numpy().reshape(shape), ref_d2)
            assert np.array_equal(site.cpu().numpy().reshape(shape), ref_s)

        edt.edt_compute_cached(g, o, d2, site, cache)
        check(rd2, rs)
        # unchanged map: the transform is skipped, the planted values stay
        d2.fill_(-5)
        site.fill_(-5)
        o.mul_(3)                               # occupied bytes 1 -> 3: still occupied
        edt.edt_compute_cached(g, o, d2, site, cache)
        check(np.full(shape, -5), np.full(shape, -5))
        # one voxel freed, one occupied: recomputed
        occ2 = occ_np.copy()
        occ2.flat[np.flatnonzero(occ2)[0]] = 0
        occ2[5, 6, 7] = 1
        o.copy_(torch.from_numpy(occ2.ravel()))
        edt.edt_compute_cached(g, o, d2, site, cache)
        r2 = oracle_lib.edt(occ2)
        check(*r2)
        # graph replays: alternate between two maps and an unchanged repeat
        gr = torch.cuda.CUDAGraph()
        edt.edt_compute_cached(g, o, d2, site, cache)
        torch.cuda.synchronize()
        with torch.cuda.graph(gr, capture_error_mode="thread_local"):
            edt.edt_compute_cached(g, o, d2, site, cache)
        for rep, (m, ref) in enumerate([(occ_np, (rd2, rs)), (occ_np, (rd2, rs)), (occ2, r2)]):
            o.copy_(torch.from_numpy(m.ravel()))
            gr.replay()
            check(*ref)
        edt.edt_cache_reset(g, cache)
        d2.fill_(-5)
        edt.edt_compute_cached(g, o, d2, site, cache)   # a reset cache computes again
        check(*r2)


LEAN_SHAPES = [(128, 64, 64), (97, 33, 65), (33, 256, 128), (32, 255, 200), (31, 1, 256), (64, 31, 127),
               (96, 256, 64), (1, 40, 64), (128, 2, 300)]


@pytest.mark.parametrize("shape", LEAN_SHAPES)
def test_lean_tiles_sparse_slices_and_rows(oracle_lib, shape):
    """Maps for the 64-column tiles (up to 128 slices and 256 rows): sites in a
    few slices only (z bands with no site, one site, or a chain the seams
    consume), sites in a few rows only (xy bands with 0-2 sites), and a dense
    map (long pop chains)."""
    nz, ny, nx = shape
    g = np.random.Generator(np.random.PCG64(nz * 7 + ny * 3 + nx))
    occ = np.zeros(shape, np.uint8)
    for z in g.choice(nz, size=min(nz, 5), replace=False):
        occ[z, g.integers(0, ny, 3), g.integers(0, nx, 3)] = 1
    assert_same(occ, oracle_lib, "few slices")
    occ = np.zeros(shape, np.uint8)
    for z in range(nz):
        for y in g.choice(ny, size=min(ny, 2), replace=False):
            occ[z, y, g.integers(0, nx, 2)] = 1
    assert_same(occ, oracle_lib, "few rows")
    assert_same(inputs.random_grid(shape, 0.3, nz + ny + nx), oracle_lib, "dense")
    assert_same_many(occ, oracle_lib, "few rows")
    assert_same_many(inputs.random_grid(shape, 0.3, nz + ny + nx), oracle_lib, "dense")


@pytest.mark.parametrize("nx", [256, 200, 300])
def test_lean_xy_equidistant_columns(oracle_lib, nx):
    """Rows whose two nearest occupied columns are equally far from many
    columns (pairs c - a, c + a, some straddling a 64-column tile boundary,
    some with the left one outside the tile): the smaller column must win, also
    where the xy stacks keep only |x - x'| (maps of at most 256 columns) and the
    side is recovered from the row; and rows with one occupied column, whose
    left side is empty."""
    nz, ny = 6, 96
    g = np.random.Generator(np.random.PCG64(nx))
    occ = np.zeros((nz, ny, nx), np.uint8)
    for z in range(nz):
        for y in range(ny):
            if y % 14 == 3:
                continue   # empty rows between
            if y % 14 == 10:
                # one occupied column, at an odd position p: column (p - 1) / 2
                # is p - x = x + 1 away with nothing on its left
                occ[z, y, 2 * ((y * 3 + z) % ((nx - 1) // 2)) + 1] = 1
                continue
            a = 1 + (y * 5 + z) % 40
            c = int(g.integers(a, nx - a))
            if y % 5 == 0:
                c = 64 * int(g.integers(1, max(2, nx // 64))) + (y % 3) - 1   # around a tile seam
                c = min(max(c, a), nx - 1 - a)
            occ[z, y, c - a] = 1
            occ[z, y, c + a] = 1
            if y % 4 == 1:
                occ[z, y, min(nx - 1, c + a + 70)] = 1   # a farther one, another tile
    say(f"[edt] equidistant columns nx={nx}")
    assert_same(occ, oracle_lib, f"equidistant nx={nx}")
    assert_same_many(occ, oracle_lib, f"equidistant nx={nx}")
