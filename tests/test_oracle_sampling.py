"""Pins for the two oracle routines that the accuracy figures rest on:

* the exact kernel rows (K W)[rows, :], the direct definition used for the
  sampled-row accuracy eps_f = |K~W - KW|_F / |KW|_F of Section 5, checked
  against a dense numpy kernel matrix for both kernels;
* the row sample of each node's ID (the sampling module of Section 3.1, under
  the reading that keeps the whole far field when it is small and otherwise
  takes the points of the nearest far clusters plus a seeded remainder),
  checked by brute force: the sample lies in the node's far field, has no
  duplicate, has the stated size, starts with the points of the far clusters
  nearest by centroid distance, and fills up with the smallest SplitMix64 keys
  (the generator from its published definition, recomputed here with numpy).

A plausible slip in either routine (a wrong kernel argument or row index,
farthest instead of nearest clusters, a duplicate row, a missed ancestor's
far list) fails one of these checks.
"""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.helpers import dense_kernel, rel

M64 = np.uint64((1 << 64) - 1)


def _mix64(z):
    """SplitMix64 finalizer (Steele, Lea, Flood, OOPSLA 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (np.asarray(z, np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & M64
        return z ^ (z >> np.uint64(31))


@pytest.mark.parametrize("kernel,h", [(wl.KERNEL_GAUSSIAN, 0.4), (wl.KERNEL_LAPLACE, 1.5)])
def test_exact_rows_equal_dense_kernel_product(kernel, h):
    w = wl.small("rows", N=1800, d=3, m=40, kernel=kernel, h=h, seed=31)
    X = wl.gen_points(w)
    H = OracleH2.from_workload(w, X)
    W = wl.gen_w(w, Q=7)
    rows = np.random.default_rng(3).choice(w.N, 50, replace=False)
    got = H.exact_rows(rows, W)
    ref = dense_kernel(X[rows], kernel, h, X) @ W
    assert rel(got, ref) <= 1e-13
    # a row of K W is the kernel row times W (original point order)
    np.testing.assert_allclose(got[0], dense_kernel(X[rows[:1]], kernel, h, X)[0] @ W, rtol=1e-12, atol=1e-13)


def _far_field(H, a):
    """Tree positions of F(a): every far partner of a and of its ancestors."""
    nodes = []
    x = a
    while x >= 0:
        nodes += [int(b) for b in H.far_col[H.far_ptr[x]:H.far_ptr[x + 1]]]
        x = int(H.parent[x])
    return nodes


def _expected_sample(H, a, S, seed):
    nodes = _far_field(H, a)
    total = int(sum(H.size[b] for b in nodes))
    if total <= S:
        return np.sort(np.concatenate([np.arange(H.start[b], H.start[b] + H.size[b]) for b in nodes])
                       if nodes else np.zeros(0, np.int64))
    cen = H.centroid
    order = sorted(nodes, key=lambda b: (float(np.linalg.norm(cen[a] - cen[b])), b))
    near_part, rest = [], []
    for b in order:
        for p in range(int(H.start[b]), int(H.start[b] + H.size[b])):
            (near_part if len(near_part) < S // 2 else rest).append(p)
    rest = np.asarray(rest, np.int64)
    base = _mix64(_mix64(np.uint64(seed)) ^ np.uint64(a))
    keys = _mix64(base ^ H.perm[rest].astype(np.uint64))
    pick = rest[np.lexsort((rest, keys))][:S - len(near_part)]
    return np.sort(np.concatenate([np.asarray(near_part, np.int64), pick]))


@pytest.mark.parametrize("w", [
    wl.small("samp_u3", N=3000, d=3, m=40, sample_rows=300, seed=41),
    wl.small("samp_mix", N=2500, d=8, points="mixture", m=50, h=1.0, sample_rows=512, seed=42),
    wl.small("samp_hss", N=2000, d=3, m=32, adm=wl.ADM_HSS, sample_rows=250, seed=43),
], ids=lambda w: w.name)
def test_row_sample_brute_force(w):
    H = OracleH2.from_workload(w, wl.gen_points(w))
    S = w.sample_rows
    n_sampled = 0
    for a in range(1, H.n_nodes):
        got = H.row_sample(a)
        far = set(p for b in _far_field(H, a) for p in range(int(H.start[b]), int(H.start[b] + H.size[b])))
        assert len(set(got.tolist())) == len(got), f"duplicate rows at node {a}"
        assert set(got.tolist()) <= far, f"row outside the far field at node {a}"
        assert len(got) == min(S, len(far))
        assert np.all(np.diff(got) > 0)
        if len(far) > S:
            n_sampled += 1
        np.testing.assert_array_equal(got, _expected_sample(H, a, S, w.sample_seed), err_msg=f"node {a}")
    assert n_sampled > 0, "the case never reaches the sampling branch"


def test_row_sample_nearest_clusters_come_first():
    """In the sampling branch, the S/2 rows taken by distance are the points
    of the nearest far clusters: a node's nearest far partner is always fully
    in its sample when it holds at most S/2 points."""
    w = wl.small("samp_near", N=4000, d=2, m=25, sample_rows=200, seed=44)
    H = OracleH2.from_workload(w, wl.gen_points(w))
    checked = 0
    for a in range(1, H.n_nodes):
        nodes = _far_field(H, a)
        if sum(int(H.size[b]) for b in nodes) <= w.sample_rows:
            continue
        d = [float(np.linalg.norm(H.centroid[a] - H.centroid[b])) for b in nodes]
        nearest = nodes[int(np.argmin(d))]
        farthest = nodes[int(np.argmax(d))]
        got = set(H.row_sample(a).tolist())
        if H.size[nearest] <= w.sample_rows // 2:
            assert set(range(int(H.start[nearest]), int(H.start[nearest] + H.size[nearest]))) <= got
            checked += 1
        # the farthest cluster is reached only by the keyed remainder: not all of it is taken
        if H.size[farthest] > 8 and len(nodes) > 4:
            assert not set(range(int(H.start[farthest]), int(H.start[farthest] + H.size[farthest]))) <= got
    assert checked > 10


def test_exact_rows_from_points_alone():
    """The points-only entry (no compression) gives the same exact rows."""
    from oracle import oracle as orc
    w = wl.small("rows_pts", N=900, d=5, points="normal", m=30, kernel=wl.KERNEL_LAPLACE, h=2.0, seed=32)
    X = wl.gen_points(w)
    W = wl.gen_w(w, Q=3)
    rows = np.arange(0, w.N, 37)
    got = orc.exact_rows(X, w.kernel, w.h, rows, W)
    assert rel(got, dense_kernel(X[rows], w.kernel, w.h, X) @ W) <= 1e-13
    np.testing.assert_array_equal(got, OracleH2.from_workload(w, X).exact_rows(rows, W))
