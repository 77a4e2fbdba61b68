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
    # the paper's high-d structure: two-means tree, budget admissibility (H^2-b)
    wl.small("tm_budget", N=1500, d=8, points="mixture", m=40, h=1.0, adm=wl.ADM_BUDGET, budget=0.1,
             part=wl.PART_TWO_MEANS),
    wl.small("tm_distance", N=1000, d=5, points="normal", m=32, h=2.0, part=wl.PART_TWO_MEANS),
    wl.small("budget_u3", N=1200, d=3, m=20, adm=wl.ADM_BUDGET, budget=0.05),
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
    if w.part != wl.PART_MEDIAN:
        pytest.skip("two-means tree (tests/test_oracle_highd.py)")
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

    near_leaf = budget_near_relation(w, H) if w.adm == wl.ADM_BUDGET else None

    def adm(a, b):
        if a == b:
            return False
        if w.adm == wl.ADM_HSS:
            return True
        if w.adm == wl.ADM_BUDGET:
            return not near_leaf[np.ix_(leaves_below(H, a), leaves_below(H, b))].any()
        dist = np.linalg.norm(H.centroid[a] - H.centroid[b])
        return w.tau * dist > 2 * H.radius[a] + 2 * H.radius[b]

    for a, b, _ in H.far_pairs():
        assert adm(a, b)
        # maximal: the parents were not admissible (else the pair would sit higher)
        pa, pb = H.parent[a], H.parent[b]
        assert pa == pb or not adm(pa, pb)
    for a, b, _ in H.near_pairs():
        assert not adm(a, b)


def leaves_below(H, a):
    """Leaf indices (0-based among the leaves, in node order) below node a."""
    first = 2 ** H.L - 1
    lv = [x - first for x in range(first, H.n_nodes)
          if x == a or _is_ancestor(H, a, x)]
    return np.array(lv, dtype=np.int64)


def _is_ancestor(H, a, x):
    while x > 0:
        x = int(H.parent[x])
        if x == a:
            return True
    return False


def budget_near_relation(w, H):
    """Near relation between leaves under the budget reading, by brute force:
    each leaf with itself and its floor(budget * #leaves) nearest leaves by
    centroid distance (ties by node number), made symmetric."""
    first, nl = 2 ** H.L - 1, 2 ** H.L
    C = H.centroid[first:first + nl]
    kb = min(int(np.floor(w.budget * nl)), nl - 1)
    near = np.eye(nl, dtype=bool)
    for x in range(nl):
        dist = np.sqrt(((C - C[x]) ** 2).sum(1))
        order = [y for y in np.lexsort((np.arange(nl), dist)) if y != x][:kb]
        near[x, order] = True
        near[order, x] = True
    return near


def test_budget_near_lists_are_the_relation():
    w = CASES[5]
    H = OracleH2.from_workload(w, wl.gen_points(w))
    near_leaf = budget_near_relation(w, H)
    first = 2 ** H.L - 1
    got = np.zeros_like(near_leaf)
    for a, b, _ in H.near_pairs():
        got[a - first, b - first] = True
    assert np.array_equal(got, near_leaf)


def test_hss_far_is_sibling():
    w = CASES[3]
    H = OracleH2.from_workload(w, wl.gen_points(w))
    for a in range(1, H.n_nodes):
        sib = a + 1 if a % 2 == 1 else a - 1
        assert H.far_col[H.far_ptr[a]:H.far_ptr[a + 1]].tolist() == [sib]
    for a, b, _ in H.near_pairs():
        assert a == b
