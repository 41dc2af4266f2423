"""GPU parity of edt_clear, edt_insert_points, edt_insert_links and
edt_query_spheres against the CPU oracle: bit-exact occupancy bytes and
bit-exact 64-byte query records (the float op order is fixed by the
interface, so floats must agree bit for bit too)."""
import numpy as np
import pytest
import torch

from paper_2407_02363_amd import edt, inputs
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def test_clear_any_alignment():
    for (nx, ny, nz), off in [((1, 1, 1), 0), ((15, 1, 1), 1), ((16, 1, 1), 0), ((17, 1, 1), 3),
                              ((1000, 1, 1), 7), ((64, 64, 1), 0), ((101, 99, 10), 5)]:
        n = nx * ny * nz
        say(f"[clear] n={n} off={off}")
        buf = torch.full((n + 32,), 0xAB, dtype=torch.uint8, device=dev())
        g = inputs.Grid(nx, ny, nz)
        view = buf[off:off + n]
        edt.edt_clear(g, view)
        torch.cuda.synchronize()
        h = buf.cpu().numpy()
        assert (h[off:off + n] == 0).all()
        assert (h[:off] == 0xAB).all() and (h[off + n:] == 0xAB).all()


def test_insert_points_cycle_frame(oracle_lib):
    ci = inputs.cycle_inputs(1, n_frames=2)
    g = ci.grid
    for k, pts in enumerate(ci.frames):
        say(f"[insert points] frame {k}")
        occ = torch.zeros(g.n, dtype=torch.uint8, device=dev())
        edt.edt_insert_points(g, occ, to_dev(pts), to_dev(ci.T_map_cam))
        ref = np.zeros(g.shape, np.uint8)
        oracle_lib.insert_points(g, ref, pts, ci.T_map_cam)
        assert np.array_equal(occ.cpu().numpy().reshape(g.shape), ref)


def test_insert_points_edge_cases_and_exclude(oracle_lib):
    g = inputs.Grid(40, 30, 20, (-0.11, 0.07, 0.0), 0.013)
    r = inputs.rng(5)
    pts = r.uniform(-0.4, 0.8, size=(50000, 3)).astype(np.float32)
    # exact voxel faces, NaN, inf, off-map
    faces = (np.array(g.origin) + r.integers(0, 41, size=(2000, 3)) * g.voxel).astype(np.float32)
    pts = np.concatenate([pts, faces, np.array([[np.nan, 0, 0], [0, np.inf, 0],
                                                [-np.inf, 0, 0], [1e30, 0, 0]], np.float32)])
    R = inputs.rot_z(0.3) @ inputs.rot_x(-1.1)
    for T in [inputs.pose12(np.eye(3), np.zeros(3)), inputs.pose12(R, [0.05, -0.02, 0.1])]:
        excl = inputs.random_grid(g.shape, 0.3, 8)
        for ex in [None, excl]:
            say(f"[insert points] edge cases exclude={ex is not None}")
            occ = torch.zeros(g.n, dtype=torch.uint8, device=dev())
            edt.edt_insert_points(g, occ, to_dev(pts), to_dev(T),
                                  exclude=None if ex is None else to_dev(ex.ravel()))
            ref = np.zeros(g.shape, np.uint8)
            oracle_lib.insert_points(g, ref, pts, T, exclude=ex)
            assert np.array_equal(occ.cpu().numpy().reshape(g.shape), ref)


def test_insert_points_or_semantics(oracle_lib):
    g = inputs.Grid(32, 32, 32, (0, 0, 0), 0.01)
    pre = inputs.random_grid(g.shape, 0.01, 4)
    pts = inputs.rng(2).uniform(0, 0.32, size=(3000, 3)).astype(np.float32)
    T = inputs.pose12(np.eye(3), np.zeros(3))
    occ = to_dev(pre.ravel().copy())
    edt.edt_insert_points(g, occ, to_dev(pts), to_dev(T))
    edt.edt_insert_points(g, occ, to_dev(pts), to_dev(T))
    ref = pre.copy()
    oracle_lib.insert_points(g, ref, pts, T)
    assert np.array_equal(occ.cpu().numpy().reshape(g.shape), ref)


@pytest.mark.parametrize("mask", [0xFF, 0x0F, 0xF0, 0x01, 0x80, 0x00, 0x5A])
def test_insert_links(oracle_lib, mask):
    ci = inputs.cycle_inputs(2, n_frames=1)
    g = ci.grid
    for qi in range(2):
        say(f"[insert links] mask={mask:#x} state {qi}")
        q = ci.joint_states[qi]
        poses = ci.robot.poses12(q)
        occ = torch.zeros(g.n, dtype=torch.uint8, device=dev())
        edt.edt_insert_links(g, occ, to_dev(ci.link_pts), ci.link_off, to_dev(poses), mask)
        ref = np.zeros(g.shape, np.uint8)
        oracle_lib.insert_links(g, ref, ci.link_pts, ci.link_off, poses, mask)
        assert np.array_equal(occ.cpu().numpy().reshape(g.shape), ref)


def run_query(g, d2, site, C, r):
    out = edt.new_query_out(len(r), dev())
    edt.edt_query_spheres(g, to_dev(d2.ravel()), to_dev(site.ravel()), to_dev(C), to_dev(r), out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def test_query_cycle_and_edges(oracle_lib):
    ci = inputs.cycle_inputs(3, n_frames=1)
    g = ci.grid
    occ = np.zeros(g.shape, np.uint8)
    oracle_lib.insert_points(g, occ, ci.frames[0], ci.T_map_cam)
    d2, site = oracle_lib.edt(occ)
    r = inputs.rng(11)
    C = np.concatenate([
        inputs.sphere_centres(ci.robot, ci.joint_states[0], ci.sphere_links, ci.sphere_local),
        r.uniform(-0.1, 2.7, size=(500, 3)).astype(np.float32),                # some outside
        (r.integers(0, 128, size=(200, 3)) * g.voxel).astype(np.float32),     # exact faces
        np.array([[0.005, 0.005, 0.005], [2.555, 2.555, 1.275], [np.nan, 1, 1]], np.float32),
    ])
    rad = r.uniform(0.02, 0.2, size=C.shape[0]).astype(np.float32)
    say(f"[query] {C.shape[0]} centres")
    got = run_query(g, d2, site, C, rad)
    ref = oracle_lib.query_spheres(g, d2, site, C, rad)
    bad = np.flatnonzero((got != ref).any(1))
    assert bad.size == 0, f"{bad.size} records differ, first {bad[:5]}: {got[bad[:1]]} vs {ref[bad[:1]]}"


def test_query_empty_and_thin_maps(oracle_lib):
    for shape in [(5, 6, 7), (1, 1, 9), (4, 1, 1)]:
        g = inputs.Grid(shape[2], shape[1], shape[0], (0.0, 0.0, 0.0), 0.1)
        for occ in [np.zeros(shape, np.uint8), inputs.random_grid(shape, 0.2, 1)]:
            d2, site = oracle_lib.edt(occ)
            C = inputs.rng(2).uniform(-0.05, 0.95, size=(64, 3)).astype(np.float32)
            rad = np.full(64, 0.05, np.float32)
            say(f"[query] thin {shape} occupied={int(occ.sum())}")
            got = run_query(g, d2, site, C, rad)
            assert np.array_equal(got, oracle_lib.query_spheres(g, d2, site, C, rad))


def test_clear_insert_links_many(oracle_lib):
    """One clear launch and one insert launch for a batch of joint states:
    every map whose gate is set equals the oracle's ClearMap + UpdateLinks for
    its own state (its old bytes gone), every map whose gate is 0 keeps its
    bytes; without gates every map is rebuilt.  Maps at odd byte offsets
    exercise the clear's unaligned head and tail."""
    st = inputs.self_map_setup()
    g = st.grid
    S = 7
    qs = inputs.random_joint_states(S, 41)
    poses = np.stack([st.robot.poses12(q) for q in qs]).astype(np.float32)
    refs = []
    for q in qs:
        ref = np.zeros(g.shape, np.uint8)
        oracle_lib.insert_links(g, ref, st.link_pts, st.link_off, st.robot.poses12(q), st.mask)
        refs.append(ref)
    buf = torch.empty(S * (g.n + 3) + 16, dtype=torch.uint8, device=dev())
    occs = [buf[1 + j * (g.n + 3):1 + j * (g.n + 3) + g.n] for j in range(S)]
    gates = torch.tensor([1, 0, 1, 1, 0, 0, 1], dtype=torch.int32, device=dev())
    pts = to_dev(st.link_pts)
    pd = to_dev(poses)
    for tag, gt in (("gated", gates), ("all", None)):
        buf.fill_(0xAB)
        say(f"[links many] {tag}")
        edt.edt_clear_insert_links_many(g, occs, pts, st.link_off, pd, st.mask, gt)
        torch.cuda.synchronize()
        on = gates.cpu().numpy() if gt is not None else np.ones(S, np.int32)
        host = buf.cpu().numpy()
        for j in range(S):
            got = occs[j].cpu().numpy().reshape(g.shape)
            if on[j]:
                assert np.array_equal(got, refs[j]), (tag, j)
            else:
                assert (got == 0xAB).all(), (tag, j)
        # the bytes between and around the maps are never written
        gaps = np.concatenate([host[:1]] + [host[1 + j * (g.n + 3) + g.n:1 + (j + 1) * (g.n + 3)]
                                            for j in range(S)])
        assert (gaps == 0xAB).all(), tag


def test_query_spheres_many(oracle_lib):
    """One launch for the sphere queries of several maps, each with its own
    grid, centres, radii and count: record (j, k) equals the oracle's query of
    map j at centre k, inside, outside and on the border of the map, on an
    empty map, and with a map that has no spheres."""
    r = inputs.rng(12)
    shapes = [(128, 256, 256), (40, 70, 130), (16, 9, 300), (64, 64, 64), (8, 8, 8)]
    counts = [70, 33, 5, 0, 64]
    grids, maps_occ, d2s, sites, cs, rs, outs, refs = [], [], [], [], [], [], [], []
    for j, (sh, m) in enumerate(zip(shapes, counts)):
        g = inputs.Grid(sh[2], sh[1], sh[0], (0.1 * j, -0.2, 0.05), 0.01 + 0.002 * j)
        occ = inputs.random_grid(sh, 0.0005 * j, 60 + j)   # map 0 is empty
        d2, site = oracle_lib.edt(occ)
        ext = np.array([g.nx, g.ny, g.nz]) * g.voxel
        C = (np.array(g.origin) + r.uniform(-0.1, 1.1, size=(m, 3)) * ext).astype(np.float32)
        if m >= 2:
            C[-2:] = np.array(g.origin, np.float32) + np.float32(0.5 * g.voxel)
            C[-1] += (ext - g.voxel).astype(np.float32)
        rad = r.uniform(0.02, 0.2, size=m).astype(np.float32)
        grids.append(g)
        maps_occ.append(to_dev(occ.ravel()))
        d2s.append(to_dev(d2.ravel()))
        sites.append(to_dev(site.ravel()))
        cs.append(to_dev(C.reshape(m, 3)))
        rs.append(to_dev(rad))
        outs.append(torch.full((max(m, 1), edt.SPHERE_RESULT_WORDS), -1, dtype=torch.int32, device=dev()))
        refs.append(oracle_lib.query_spheres(g, d2, site, C, rad))
    maps = edt.batch_maps(grids, maps_occ, d2s, sites)
    edt.edt_query_spheres_many(maps, cs, rs, [o[:max(c, 0) or 1] for o, c in zip(outs, counts)])
    torch.cuda.synchronize()
    for j, m in enumerate(counts):
        got = outs[j].cpu().numpy().view(np.uint32)
        if m:
            assert np.array_equal(got[:m], refs[j]), j
        else:
            assert (got == 0xFFFFFFFF).all(), "a map without spheres is left alone"


def test_clear_insert_points_many(oracle_lib):
    """One clear launch and one insertion launch for maps of different grids,
    clouds and poses (an empty cloud among them): every map equals the
    oracle's ClearMap + Insert(Point_Cloud) of its own cloud, whatever it
    held before, at odd byte offsets."""
    shapes = [(128, 96, 200), (64, 64, 64), (40, 70, 130), (9, 300, 16)]
    grids, occs, clouds, poses, refs = [], [], [], [], []
    buf = torch.full((sum(int(np.prod(sh)) + 3 for sh in shapes) + 16,), 0xAB, dtype=torch.uint8, device=dev())
    off = 1
    for j, sh in enumerate(shapes):
        ci = inputs.cycle_inputs(j, n_frames=1, grid=inputs.Grid(sh[2], sh[1], sh[0], (1.0, 0.9, 0.0), 0.02))
        g = ci.grid
        pts = ci.frames[0][::(j + 1) * 3] if j != 1 else np.zeros((0, 3), np.float32)
        ref = np.zeros(g.shape, np.uint8)
        oracle_lib.insert_points(g, ref, pts, ci.T_map_cam)
        n = g.n
        grids.append(g)
        occs.append(buf[off:off + n])
        off += n + 3
        clouds.append(to_dev(np.ascontiguousarray(pts, np.float32).reshape(-1, 3)))
        poses.append(to_dev(np.asarray(ci.T_map_cam, np.float32)))
        refs.append(ref)
    say(f"[points many] {len(shapes)} maps, {sum(c.shape[0] for c in clouds)} points")
    edt.edt_clear_insert_points_many(grids, occs, clouds, poses)
    torch.cuda.synchronize()
    for j, g in enumerate(grids):
        assert np.array_equal(occs[j].cpu().numpy().reshape(g.shape), refs[j]), j
    assert refs[0].any() and not refs[1].any()
