"""Pins for the oracle's cluster tree and interaction lists (Section 3.1 tree
construction / interaction computation; admissibility of Section 2.1; HSS of
Section 4.1), checked by brute force on small point sets."""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2

CASES = [
    wl.small("u3", N=1000, d=3, m=32),
    wl.small("u2_ragged", N=777, d=2, m=20),
    wl.small("mix8", N=1500, d=8, points="mixture", m=40, h=1.0),
    wl.small("hss", N=900, d=3, m=30, adm=wl.ADM_HSS),
    wl.small("single", N=50, d=3, m=64),
]


@pytest.fixture(scope="module", params=CASES, ids=[c.name for c in CASES])
def built(request):
    w = request.param
    X = wl.gen_points(w)
    return w, X, OracleH2.from_workload(w, X)


def test_tree_is_perfect_partition(built):
    w, X, H = built
    N = w.N
    assert sorted(H.perm.tolist()) == list(range(N))
    # minimal depth with leaves of at most m points
    L = H.L
    assert -(-N // (1 << L)) <= w.m
    assert L == 0 or -(-N // (1 << (L - 1))) > w.m
    assert H.n_nodes == 2 ** (L + 1) - 1
    assert H.start[0] == 0 and H.size[0] == N and H.parent[0] == -1
    for a in range(H.n_nodes):
        assert H.level[a] == int(np.floor(np.log2(a + 1)))
        if H.level[a] == L:
            assert H.left[a] == -1 and H.right[a] == -1
            assert 1 <= H.size[a] <= w.m
        else:
            l, r = H.left[a], H.right[a]
            assert (l, r) == (2 * a + 1, 2 * a + 2)
            assert H.parent[l] == a and H.parent[r] == a
            assert H.start[l] == H.start[a] and H.size[l] == H.size[a] // 2
            assert H.start[r] == H.start[a] + H.size[l]
            assert H.size[l] + H.size[r] == H.size[a]


def test_split_is_median_of_widest_coordinate(built):
    w, X, H = built
    for a in range(H.n_nodes):
        if H.left[a] < 0:
            continue
        idx = H.perm[H.start[a]:H.start[a] + H.size[a]]
        pts = X[idx]
        j = int(np.argmax(pts.max(0) - pts.min(0)))  # first maximum = lowest coordinate
        order = np.lexsort((idx, pts[:, j]))           # by value, then original index
        half = len(idx) // 2
        l = H.left[a]
        left_set = set(H.perm[H.start[l]:H.start[l] + H.size[l]].tolist())
        assert left_set == set(idx[order[:half]].tolist()), f"node {a} split on coordinate {j}"


def test_geometry_matches_definition(built):
    w, X, H = built
    for a in range(H.n_nodes):
        pts = X[H.perm[H.start[a]:H.start[a] + H.size[a]]]
        c = pts.mean(0)
        np.testing.assert_allclose(H.centroid[a], c, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(H.radius[a], np.sqrt(((pts - c) ** 2).sum(1)).max(), rtol=1e-12)


def test_blocks_cover_matrix_exactly_once(built):
    w, X, H = built
    N = w.N
    cover = np.zeros((N, N), np.int16)
    for a, b, _ in H.near_pairs():
        assert H.left[a] < 0 and H.left[b] < 0, "near pairs only between leaves"
        cover[H.start[a]:H.start[a] + H.size[a], H.start[b]:H.start[b] + H.size[b]] += 1
    for a, b, _ in H.far_pairs():
        assert a != b
        cover[H.start[a]:H.start[a] + H.size[a], H.start[b]:H.start[b] + H.size[b]] += 1
    assert cover.min() == 1 and cover.max() == 1


def test_lists_are_symmetric_and_sorted(built):
    w, X, H = built
    far = set((a, b) for a, b, _ in H.far_pairs())
    near = set((a, b) for a, b, _ in H.near_pairs())
    assert all((b, a) in far for a, b in far)
    assert all((b, a) in near for a, b in near)
    for ptr, col in ((H.far_ptr, H.far_col), (H.near_ptr, H.near_col)):
        for a in range(H.n_nodes):
            seg = col[ptr[a]:ptr[a + 1]]
            assert np.all(np.diff(seg) > 0)


def test_admissibility_decisions(built):
    w, X, H = built

    def adm(a, b):
        if a == b:
            return False
        if w.adm == wl.ADM_HSS:
            return True
        dist = np.linalg.norm(H.centroid[a] - H.centroid[b])
        return w.tau * dist > 2 * H.radius[a] + 2 * H.radius[b]

    for a, b, _ in H.far_pairs():
        assert adm(a, b)
        # maximal: the parents were not admissible (else the pair would sit higher)
        pa, pb = H.parent[a], H.parent[b]
        assert pa == pb or not adm(pa, pb)
    for a, b, _ in H.near_pairs():
        assert not adm(a, b)


def test_hss_far_is_sibling():
    w = CASES[3]
    H = OracleH2.from_workload(w, wl.gen_points(w))
    for a in range(1, H.n_nodes):
        sib = a + 1 if a % 2 == 1 else a - 1
        assert H.far_col[H.far_ptr[a]:H.far_ptr[a + 1]].tolist() == [sib]
    for a, b, _ in H.near_pairs():
        assert a == b
