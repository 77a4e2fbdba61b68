"""Pins for the oracle's evaluation Y = K~ W (Section 2.1, "Evaluation") and
for the compressed matrix it evaluates: the tree walk against the dense K~
assembled from its block definition, the compression against the dense
kernel product (overall accuracy eps_f of Section 5), and invariants."""
import os

import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.helpers import dense_kernel, read_hmc1, rel

SMALL = [
    wl.small("u3", N=1000, d=3, m=32, Q=5),
    wl.small("ragged", N=777, d=2, m=20, Q=3),
    wl.small("mix8", N=1500, d=8, points="mixture", m=40, h=1.0, Q=4),
    wl.small("hss_lap", N=900, d=3, m=30, adm=wl.ADM_HSS, kernel=wl.KERNEL_LAPLACE, h=2.0, Q=6),
]


@pytest.fixture(scope="module")
def c1():
    w = wl.C1
    X = wl.gen_points(w)
    return w, X, OracleH2.from_workload(w, X)


@pytest.mark.parametrize("w", SMALL, ids=[c.name for c in SMALL])
def test_tree_walk_equals_dense_ktilde(w):
    X = wl.gen_points(w)
    H = OracleH2.from_workload(w, X)
    W = wl.gen_w(w)
    Y = H.eval(W)
    Kt = H.dense_ktilde()
    assert rel(Y, Kt @ W) <= 1e-12


def test_c1_tree_walk_and_accuracy(c1):
    w, X, H = c1
    W = wl.gen_w(w)
    Y = H.eval(W)
    Kt = H.dense_ktilde()
    assert rel(Y, Kt @ W) <= 1e-12
    K = dense_kernel(X, w.kernel, w.h)
    KW = K @ W
    eps_f = rel(Y, KW)          # overall accuracy, Section 5
    assert eps_f <= w.tol, eps_f
    # far pairs exist on at least two levels (the structure is a real H^2 one)
    levels = {int(H.level[a]) for a, _, _ in H.far_pairs()}
    assert len(levels) >= 2


def test_near_part_is_exact_kernel_on_near_blocks(c1):
    """The near part of the walk equals the exact kernel restricted to the
    near blocks; the far part approximates the rest within the tolerance."""
    w, X, H = c1
    W = wl.gen_w(w)
    Y, ph = H.eval(W, dump=True)
    K = dense_kernel(X, w.kernel, w.h)
    mask = np.zeros_like(K, dtype=bool)
    for a, b, _ in H.near_pairs():
        ia = H.perm[H.start[a]:H.start[a] + H.size[a]]
        ib = H.perm[H.start[b]:H.start[b] + H.size[b]]
        mask[np.ix_(ia, ib)] = True
    yn = np.empty_like(Y)
    yf = np.empty_like(Y)
    yn[H.perm] = ph["ynear"]
    yf[H.perm] = ph["yfar"]
    np.testing.assert_allclose(yn, (K * mask) @ W, rtol=0, atol=1e-12 * np.abs(K @ W).max())
    # the far part carries all of the approximation error, measured as in eps_f
    assert np.linalg.norm(yf - (K * ~mask) @ W) <= w.tol * np.linalg.norm(K @ W)
    np.testing.assert_array_equal(Y, yn + yf)


def test_leaf_size_at_least_n_is_dense_product():
    w = wl.small("one", N=300, d=3, m=300, Q=4)
    X = wl.gen_points(w)
    H = OracleH2.from_workload(w, X)
    assert H.n_nodes == 1 and H.n_far == 0 and H.n_near == 1
    W = wl.gen_w(w)
    K = dense_kernel(X, w.kernel, w.h)
    np.testing.assert_allclose(H.eval(W), K @ W, rtol=1e-14, atol=1e-14 * np.abs(K @ W).max())


def test_full_rank_reproduces_kernel():
    w = wl.small("full", N=512, d=3, m=16, tol=0.0, rmax=512, Q=3)
    X = wl.gen_points(w)
    H = OracleH2.from_workload(w, X)
    assert H.n_far > 0
    K = dense_kernel(X, w.kernel, w.h)
    assert rel(H.dense_ktilde(), K) <= 1e-12


def test_symmetry(c1):
    w, X, H = c1
    far = {(a, b): e for a, b, e in H.far_pairs()}
    for (a, b), e in far.items():
        assert np.array_equal(H.B_block(e, a, b), H.B_block(far[(b, a)], b, a).T)
    near = {(a, b): e for a, b, e in H.near_pairs()}
    for (a, b), e in near.items():
        assert np.array_equal(H.D_block(e, a, b), H.D_block(near[(b, a)], b, a).T)
    rng = np.random.default_rng(9)
    u, v = rng.standard_normal((w.N, 1)), rng.standard_normal((w.N, 1))
    lhs, rhs = float(u.T @ H.eval(v)), float(v.T @ H.eval(u))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(v) * w.N


def test_linearity_and_column_independence(c1):
    w, X, H = c1
    rng = np.random.default_rng(10)
    W1, W2 = rng.standard_normal((w.N, 3)), rng.standard_normal((w.N, 3))
    Y1, Y2 = H.eval(W1), H.eval(W2)
    Y = H.eval(2.0 * W1 - 0.5 * W2)
    assert rel(Y, 2.0 * Y1 - 0.5 * Y2) <= 1e-14
    Yc = H.eval(W1[:, 1:2])
    np.testing.assert_array_equal(Yc[:, 0], Y1[:, 1])


def test_skeleton_blocks_are_kernel_values(c1):
    w, X, H = c1
    for a, b, e in list(H.far_pairs())[:50]:
        sa = H.skel[H.skel_ptr[a]:H.skel_ptr[a + 1]]
        sb = H.skel[H.skel_ptr[b]:H.skel_ptr[b + 1]]
        np.testing.assert_allclose(H.B_block(e, a, b), dense_kernel(X[sa], w.kernel, w.h, X[sb]),
                                   rtol=1e-15, atol=0)


def test_file_round_trip(c1, tmp_path):
    w, X, H = c1
    path = os.path.join(tmp_path, "c1.hmc")
    H.write(path)
    f = read_hmc1(path)
    assert f["version"] == 1 and f["N"] == w.N and f["d"] == w.d and f["L"] == H.L
    assert f["kernel"] == w.kernel and f["h"] == w.h and f["tol"] == w.tol and f["m"] == w.m
    for k in ("perm", "start", "size", "parent", "left", "right", "level", "rank", "basis_off",
              "basis", "far_ptr", "far_col", "far_off", "B", "near_ptr", "near_col", "near_off",
              "D", "skel_ptr", "skel"):
        assert np.array_equal(f[k], getattr(H, k)), k


def test_row_sampling_branch_keeps_accuracy(c1):
    """With a row-sample cap below the far-field sizes (the sampling branch of
    the ID), the walk still equals its dense K~ and the overall accuracy stays
    within twice the block tolerance (sampling is a heuristic, so the bar is
    looser than for exact far-field rows)."""
    import dataclasses
    w, X, _ = c1
    ws = dataclasses.replace(w, sample_rows=512)
    H = OracleH2.from_workload(ws, X)
    far_sizes = []
    for a in range(H.n_nodes):
        tot, x = 0, a
        while x >= 0:
            tot += int(sum(H.size[H.far_col[H.far_ptr[x]:H.far_ptr[x + 1]]]))
            x = H.parent[x]
        far_sizes.append(tot)
    assert max(far_sizes) > 512
    W = wl.gen_w(w)
    Y = H.eval(W)
    assert rel(Y, H.dense_ktilde() @ W) <= 1e-12
    assert rel(Y, dense_kernel(X, w.kernel, w.h) @ W) <= 2 * w.tol
