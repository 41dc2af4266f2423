"""Pins of the CPU oracle's statistical outlier filter (Sec. III-A: the raw
cloud is filtered by each point's Euclidean distance to its neighbours):
a worked example, scipy's k-d tree neighbour search, permutation
invariance, duplicates and non-finite points."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_2407_02363_amd import inputs


def test_worked_example():
    p = np.array([[0, 0, 0], [0.003, 0, 0], [0, 0.004, 0], [1, 1, 1]], np.float32)
    keep, d, (mu, sigma, thr) = oracle.outlier_filter(p, k=2, radius=0.01, alpha=1.0)
    # neighbours: 0 -> {3 mm, 4 mm}; 1 -> {3 mm, 5 mm}; 2 -> {4 mm, 5 mm};
    # 3 has none within 1 cm, so both count as 1 cm
    assert np.allclose(d, [0.0035, 0.004, 0.0045, 0.01], rtol=1e-6)
    assert abs(mu - 0.0055) < 1e-9
    assert abs(sigma - np.sqrt(27.5e-6 / 3)) < 1e-9
    assert keep.tolist() == [1, 1, 1, 0]


def kdtree_means(p, k, r):
    t = cKDTree(p.astype(np.float64))
    dist, idx = t.query(p.astype(np.float64), k=k + 1, distance_upper_bound=r)
    dist = dist[:, 1:]                                 # drop the point itself
    dist = np.where(np.isfinite(dist), dist, r)
    return dist.mean(axis=1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_against_kdtree(seed):
    """Mean neighbour distances agree with scipy's k-d tree to float32
    rounding; the keep decision agrees wherever d is not within that
    rounding of the threshold."""
    g = inputs.rng(seed)
    # a noisy surface patch plus scattered outliers
    n = 3000
    uv = g.uniform(0, 0.08, (n, 2))
    z = 0.5 + 0.01 * np.sin(40 * uv[:, 0]) + g.normal(0, 0.0008, n)
    p = np.column_stack([uv, z]).astype(np.float32)
    out = g.choice(n, 40, replace=False)
    p[out, 2] += g.uniform(0.02, 0.2, 40).astype(np.float32)
    k, r = 8, 0.01
    keep, d, (mu, sigma, thr) = oracle.outlier_filter(p, k=k, radius=r, alpha=1.0)
    ref = kdtree_means(p, k, r)
    assert np.allclose(d, ref, rtol=2e-6, atol=1e-9)
    ref_mu, ref_sigma = ref.mean(), ref.std(ddof=1)
    assert abs(mu - ref_mu) < 1e-7 and abs(sigma - ref_sigma) < 1e-7
    clear = np.abs(ref - (ref_mu + ref_sigma)) > 1e-6
    assert np.array_equal(keep[clear].astype(bool), (ref <= ref_mu + ref_sigma)[clear])
    # the planted outliers are dropped, most surface points kept
    assert keep[out].sum() == 0 and keep.mean() > 0.8


def test_permutation_duplicates_and_nan():
    g = inputs.rng(7)
    p = g.uniform(0, 0.03, (400, 3)).astype(np.float32)
    keep, d, st = oracle.outlier_filter(p, k=5, radius=0.01, alpha=0.5)
    perm = g.permutation(400)
    keep2, d2, st2 = oracle.outlier_filter(p[perm], k=5, radius=0.01, alpha=0.5)
    assert np.array_equal(d2, d[perm]) and np.array_equal(keep2, keep[perm]) and st2 == st
    # five copies of one point: its copies are its nearest neighbours at 0
    q = np.vstack([np.repeat(p[:1], 6, axis=0), p[1:]])
    _, dq, _ = oracle.outlier_filter(q, k=5, radius=0.01, alpha=0.5)
    assert (dq[:6] == 0).all()
    # non-finite points are dropped and are nobody's neighbour
    r = p.copy()
    r[10] = [np.nan, 0, 0]
    r[11] = [np.inf, 1, 1]
    keep3, d3, _ = oracle.outlier_filter(r, k=5, radius=0.01, alpha=0.5)
    assert keep3[10] == 0 and keep3[11] == 0 and np.isnan(d3[10]) and np.isnan(d3[11])
    rest = np.delete(np.arange(400), [10, 11])
    _, d4, _ = oracle.outlier_filter(r[rest], k=5, radius=0.01, alpha=0.5)
    assert np.array_equal(d3[rest], d4)
