"""The statistical outlier filter (Sec. III-A) on the GPU against the CPU
oracle: keep mask, mean neighbour distances and the statistics bit for bit
on small clouds and on a full 640 x 480 frame, edge cases, and the filtered
frame feeding the probabilistic occupancy update."""
import numpy as np
import pytest
import torch

import oracle
from paper_2407_02363_amd import edt, inputs
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu

SCALE1, SCALE2 = 2.0 ** 40, 2.0 ** 48


def gpu_filter(p, k=8, radius=0.01, alpha=1.0):
    d = dev()
    n = p.shape[0]
    pt = torch.from_numpy(np.ascontiguousarray(p, np.float32)).to(d)
    keep = torch.full((max(n, 1),), 7, dtype=torch.uint8, device=d)[:n]
    dm = torch.zeros(max(n, 1), dtype=torch.float32, device=d)[:n]
    st = torch.zeros(3, dtype=torch.float64, device=d)
    ws = edt.new_outlier_workspace(n, d)
    edt.edt_outlier_filter(pt, keep, ws, k=k, radius=radius, alpha=alpha, mean_dist=dm, stats=st)
    torch.cuda.synchronize()
    return keep.cpu().numpy(), dm.cpu().numpy(), tuple(st.cpu().numpy().tolist())


def frame_cloud(seed, stride, frac=0.01, nan_frac=0.002):
    ci = inputs.cycle_inputs(seed, n_frames=1, grid=inputs.Grid(32, 32, 32, (1.0, 1.0, 0.0), 0.05))
    return inputs.with_outliers(ci.frames[0][::stride], frac, seed + 1, nan_frac)


@pytest.mark.parametrize("case", ["patch", "frame_sub", "k4_alpha0"])
def test_matches_oracle(case):
    if case == "patch":
        g = inputs.rng(0)
        uv = g.uniform(0, 0.08, (3000, 2))
        z = 0.5 + 0.01 * np.sin(40 * uv[:, 0]) + g.normal(0, 0.0008, 3000)
        p = np.column_stack([uv, z]).astype(np.float32)
        p[::75, 2] += 0.05
        args = dict(k=8, radius=0.01, alpha=1.0)
    elif case == "frame_sub":
        p = frame_cloud(1, 10)
        args = dict(k=8, radius=0.02, alpha=1.0)
    else:
        p = frame_cloud(2, 12)
        args = dict(k=4, radius=0.015, alpha=0.0)
    say(f"[outlier] {case}: {p.shape[0]} points {args}")
    gk, gd, gs = gpu_filter(p, **args)
    rk, rd, rs = oracle.outlier_filter(p, **args)
    assert np.array_equal(np.isnan(gd), np.isnan(rd))
    fin = ~np.isnan(rd)
    assert np.array_equal(gd[fin], rd[fin]), np.flatnonzero(gd[fin] != rd[fin])[:5]
    assert gs == rs
    assert np.array_equal(gk, rk)
    assert 0 < rk.sum() < p.shape[0]


def test_full_frame_matches_oracle():
    """The full 640 x 480 frame (307,200 points, 1% flying pixels, 0.2% NaN):
    every d_i, the statistics and every keep decision against the all-pairs
    oracle; the statistics also follow exactly from the device's own d_i."""
    ci = inputs.cycle_inputs(0, n_frames=1)
    p = inputs.with_outliers(ci.frames[0], 0.01, 5, 0.002)
    say(f"[outlier] full frame {p.shape[0]} points")
    gk, gd, (mu, sigma, thr) = gpu_filter(p)
    rk, rd, rs = oracle.outlier_filter(p)
    assert np.array_equal(np.isnan(gd), np.isnan(rd))
    fin = ~np.isnan(rd)
    assert np.array_equal(gd[fin], rd[fin]), np.flatnonzero(gd[fin] != rd[fin])[:5]
    assert (mu, sigma, thr) == rs
    assert np.array_equal(gk, rk)
    f = ~np.isnan(gd)
    d64 = gd[f].astype(np.float64)
    S1 = int(np.rint(d64 * SCALE1).astype(np.int64).sum())
    S2 = int(np.rint(d64 * d64 * SCALE2).astype(np.int64).sum())
    cnt = int(f.sum())
    mu_r = S1 / SCALE1 / cnt
    var = (S2 / SCALE2 - cnt * mu_r * mu_r) / (cnt - 1)
    assert mu == mu_r and sigma == np.sqrt(var) and thr == mu_r + 1.0 * np.sqrt(var)
    say(f"[outlier] kept {gk.mean():.4f}, mu {mu * 1e3:.3f} mm, sigma {sigma * 1e3:.3f} mm")


def test_edge_cases():
    empty = gpu_filter(np.zeros((0, 3), np.float32))
    assert empty[0].size == 0 and empty[2] == (0.0, 0.0, 0.0)
    one = gpu_filter(np.array([[0.1, 0.2, 0.3]], np.float32))
    assert one[0].tolist() == [1] and one[1][0] == np.float32(0.01)
    nan = np.full((50, 3), np.nan, np.float32)
    k, d, st = gpu_filter(nan)
    assert (k == 0).all() and np.isnan(d).all() and st == (0.0, 0.0, 0.0)
    # far-apart points: nobody has a neighbour, every d_i is the radius
    far = (np.arange(30, dtype=np.float32)[:, None] * np.float32(0.5)) * np.ones((1, 3), np.float32)
    k, d, st = gpu_filter(far)
    assert (d == np.float32(0.01)).all() and (k == 1).all() and st[1] < 1e-7


def test_clusters_sharing_table_buckets():
    """Clusters that the neighbour-search table folds onto the same buckets,
    and runs of cells that wrap round the table: the search wraps its grid
    of cells (half the radius) with a period of 16 cells per axis for 1,020
    points, so clusters 16 cells apart share buckets and a cluster around the
    origin straddles the wrap.  Every d_i and keep decision
    against the all-pairs oracle."""
    R = 0.01
    period = 16 * np.float32(R * 0.5005)
    g = inputs.rng(44)
    base = g.uniform(-0.012, 0.012, (250, 3)).astype(np.float32)
    shifts = [(0, 0, 0), (period, 0, 0), (0, period, period), (-period, -2 * period, 0)]
    p = np.concatenate([base + np.float32(s) for s in [np.array(v, np.float32) for v in shifts]])
    p = np.concatenate([p, g.uniform(-0.2, 0.2, (20, 3)).astype(np.float32)])
    say(f"[outlier] folded clusters: {p.shape[0]} points")
    gk, gd, gs = gpu_filter(p, k=8, radius=R, alpha=0.5)
    rk, rd, rs = oracle.outlier_filter(p, k=8, radius=R, alpha=0.5)
    assert np.array_equal(gd, rd), np.flatnonzero(gd != rd)[:5]
    assert gs == rs and np.array_equal(gk, rk)
    assert 0 < rk.sum() < p.shape[0]


def test_filtered_frame_feeds_logodds_update():
    ci = inputs.cycle_inputs(9, n_frames=1, grid=inputs.Grid(96, 80, 48, (0.7, 0.6, 0.0), 0.025))
    g = ci.grid
    p = inputs.with_outliers(ci.frames[0][::4], 0.02, 10, 0.002)
    rk, _, _ = oracle.outlier_filter(p, k=8, radius=0.02, alpha=1.0)
    d = dev()
    pt = torch.from_numpy(p).to(d)
    keep = torch.empty(p.shape[0], dtype=torch.uint8, device=d)
    edt.edt_outlier_filter(pt, keep, edt.new_outlier_workspace(p.shape[0], d), k=8, radius=0.02)
    L = torch.zeros(g.n, dtype=torch.int16, device=d)
    occ = torch.empty(g.n, dtype=torch.uint8, device=d)
    ws = edt.new_logodds_workspace(g, d)
    edt.edt_logodds_reset(g, L, ws)
    edt.edt_update_logodds(g, L, occ, pt, torch.from_numpy(ci.T_map_cam).to(d), ws, keep=keep)
    torch.cuda.synchronize()
    assert np.array_equal(keep.cpu().numpy(), rk)
    RL = np.zeros(g.n, np.int16)
    RO = np.zeros(g.n, np.uint8)
    oracle.update_logodds(g, RL, RO, p, ci.T_map_cam, keep=rk)
    assert np.array_equal(L.cpu().numpy(), RL) and np.array_equal(occ.cpu().numpy(), RO)
    # the filter removed voxels that the unfiltered frame would occupy
    RL2 = np.zeros(g.n, np.int16)
    RO2 = np.zeros(g.n, np.uint8)
    oracle.update_logodds(g, RL2, RO2, p, ci.T_map_cam)
    assert RO2.sum() > RO.sum()
