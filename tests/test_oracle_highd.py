"""Pins for the oracle's high-dimensional structure options: the two-means
tree (Section 3.1: two-means partitioning for d > 3) and budget
admissibility (Section 4.1: GOFMM's budget, 0.03 for H^2-b and 0 for HSS).

Two-means: the two means of every split are those of scikit-learn's Lloyd
k-means (k = 2) from the same two starting points; they are a fixed point
(each mean is the mean of the points nearer to it); the children are the
lower and upper halves along c2 - c1.  Budget: budget 0 gives exactly the
HSS lists and budget 1 gives no far pair; evaluation on these structures
equals the dense K~ of the block definition."""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.helpers import rel

TM = wl.small("tm", N=2000, d=8, points="mixture", m=40, h=1.0, part=wl.PART_TWO_MEANS)


@pytest.fixture(scope="module")
def tm():
    X = wl.gen_points(TM)
    return X, OracleH2.from_workload(TM, X)


def _start_points(P, idx):
    """The starting means of the reading: the point farthest from the
    centroid, then the point farthest from it (lowest original index on ties)."""
    c = P.mean(0)
    d0 = ((P - c) ** 2).sum(1)
    i1 = np.lexsort((idx, -d0))[0]
    d1 = ((P - P[i1]) ** 2).sum(1)
    i2 = np.lexsort((idx, -d1))[0]
    return P[i1], P[i2]


def test_two_means_centers_are_lloyd_kmeans(tm):
    from sklearn.cluster import KMeans
    X, H = tm
    checked = 0
    for a in range(H.n_nodes):
        if H.left[a] < 0:
            continue
        idx = H.perm[H.start[a]:H.start[a] + H.size[a]]
        P = X[idx]
        c1, c2 = H.split_centers(a)
        s1, s2 = _start_points(P, idx)
        km = KMeans(n_clusters=2, init=np.stack([s1, s2]), n_init=1, max_iter=100, tol=0.0,
                    algorithm="lloyd").fit(P)
        np.testing.assert_allclose(km.cluster_centers_[0], c1, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(km.cluster_centers_[1], c2, rtol=1e-10, atol=1e-10)
        checked += 1
    assert checked == H.n_nodes // 2


def test_two_means_centers_are_a_fixed_point_and_split_is_the_median_cut(tm):
    X, H = tm
    for a in range(H.n_nodes):
        if H.left[a] < 0:
            continue
        idx = H.perm[H.start[a]:H.start[a] + H.size[a]]
        P = X[idx]
        c1, c2 = H.split_centers(a)
        g = ((P - c2) ** 2).sum(1) < ((P - c1) ** 2).sum(1)
        assert 0 < g.sum() < len(P)
        np.testing.assert_allclose(P[~g].mean(0), c1, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(P[g].mean(0), c2, rtol=1e-12, atol=1e-12)
        key = P @ (c2 - c1)
        l = H.left[a]
        left = np.isin(idx, H.perm[H.start[l]:H.start[l] + H.size[l]])
        assert left.sum() == len(P) // 2
        assert key[left].max() <= key[~left].min()


def test_median_tree_has_no_two_means_centers():
    w = wl.small("m", N=500, d=3, m=32)
    H = OracleH2.from_workload(w, wl.gen_points(w))
    assert all(H.split_centers(a) is None for a in range(H.n_nodes))


def _lists(H):
    far = [(a, b) for a, b, _ in H.far_pairs()]
    near = [(a, b) for a, b, _ in H.near_pairs()]
    return far, near


def test_budget_zero_is_hss_and_budget_one_is_dense():
    base = dict(N=1200, d=8, points="mixture", m=30, h=1.0, part=wl.PART_TWO_MEANS)
    X = wl.gen_points(wl.small("b", **base))
    h0 = OracleH2.from_workload(wl.small("b", adm=wl.ADM_BUDGET, budget=0.0, **base), X)
    hs = OracleH2.from_workload(wl.small("b", adm=wl.ADM_HSS, **base), X)
    assert _lists(h0) == _lists(hs)
    h1 = OracleH2.from_workload(wl.small("b", adm=wl.ADM_BUDGET, budget=1.0, **base), X)
    far, near = _lists(h1)
    nl = 2 ** h1.L
    assert far == [] and len(near) == nl * nl


@pytest.mark.parametrize("w", [
    wl.small("tm_budget", N=1500, d=8, points="mixture", m=40, h=1.0, adm=wl.ADM_BUDGET, budget=0.1,
             part=wl.PART_TWO_MEANS, Q=5),
    wl.small("budget_lap", N=1000, d=5, points="normal", m=32, h=2.0, adm=wl.ADM_BUDGET, budget=0.05,
             kernel=wl.KERNEL_LAPLACE, part=wl.PART_TWO_MEANS, Q=3),
], ids=["tm_budget", "budget_lap"])
def test_tree_walk_equals_dense_ktilde_on_budget_structures(w):
    X = wl.gen_points(w)
    H = OracleH2.from_workload(w, X)
    W = wl.gen_w(w)
    Y = H.eval(W)
    assert rel(Y, H.dense_ktilde() @ W) <= 1e-12
