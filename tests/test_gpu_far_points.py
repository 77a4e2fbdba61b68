"""Matrix-free far field on the GPU: with HM_FAR_FROM_POINTS the FP64
task-graph launch computes every far (coupling) block B_ab =
K(X[skel_a], X[skel_b]) (Section 2.1: the coupling block of the ID-based H2
representation is the kernel matrix of the two nodes' skeletons) inside its
product tiles instead of reading it from the device store.  Checked against
the CPU FP64 oracle's tree walk (which reads the blocks it computed at
compression) to the FP64 bar, and against the stored-block path; the only
differences are the device's exp/sqrt rounding and the summation order."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.helpers import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "c1": wl.C1,
    "ragged": wl.small("ragged", N=777, d=2, m=20, Q=3),
    "mix8": wl.small("mix8", N=3000, d=8, points="mixture", m=50, h=1.0, Q=37),
    "hss_lap": wl.small("hss_lap", N=2500, d=3, m=70, adm=wl.ADM_HSS, kernel=wl.KERNEL_LAPLACE,
                        h=2.0, rmax=70, Q=20),
    "deep_small_leaves": wl.small("deep", N=2048, d=3, m=8, Q=4, rmax=8),
    "d15": wl.small("d15", N=1500, d=15, points="normal", m=100, adm=wl.ADM_HSS,
                    kernel=wl.KERNEL_LAPLACE, h=4.0, tol=1e-4, rmax=100, Q=9),
    # above 15 dimensions the tiles read their points from global memory
    "d28": wl.small("d28", N=1800, d=28, points="normal", m=100, adm=wl.ADM_HSS,
                    kernel=wl.KERNEL_LAPLACE, h=4.0, tol=1e-4, rmax=100, Q=11),
    # leaves of up to 188 points and ranks up to 200: blocks taller than one
    # 128-row tile, whose second tile starts at row 128 of the block
    "tall_tiles": wl.small("tall", N=3000, d=3, m=256, adm=wl.ADM_HSS, kernel=wl.KERNEL_LAPLACE,
                           h=1.0, tol=1e-10, rmax=200, Q=5),
    "tall_tiles_d28": wl.small("tall28", N=3000, d=28, points="normal", m=256, adm=wl.ADM_HSS,
                               kernel=wl.KERNEL_LAPLACE, h=4.0, tol=1e-8, rmax=200, Q=5),
    "tm_budget": wl.small("tm_budget", N=3000, d=8, points="mixture", m=50, h=1.0, adm=wl.ADM_BUDGET,
                          budget=0.1, part=wl.PART_TWO_MEANS, Q=24),
}
_built = {}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hmx():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1812_07152_amd as hmx
    return hmx


def built(name):
    if name not in _built:
        w = CASES[name]
        X = wl.gen_points(w)
        _built[name] = (w, X, OracleH2.from_workload(w, X))
    return _built[name]


def run(hmx, M, W, flags):
    Wd = torch.from_numpy(W).to("cuda", torch.float64)
    Yd = torch.full_like(Wd, float("nan"))
    hmx.hm_eval(M, Wd, Yd, flags=flags)
    hmx.hm_check(M)
    return Yd.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_far_from_points_matches_oracle(hmx, name):
    w, X, H = built(name)
    assert H.stats()["E_B"] > 0, "the case must have far blocks"
    M = hmx.hm_load_compressed_mem(H, 0)
    hmx.hm_set_points(M, X, w.kernel, w.h)
    both = hmx.HM_NEAR_FROM_POINTS | hmx.HM_FAR_FROM_POINTS
    for Q in (w.Q, 40, 300):  # 40: the 64-column tile, run at 128 columns in this mode
        _say(f"[far-points] case={name} N={w.N} d={w.d} Q={Q}")
        W = wl.gen_w(w, Q=Q, seed=600 + Q)
        Yref = H.eval(W)
        Ys = run(hmx, M, W, 0)  # stored blocks, same launch otherwise
        tol = 1e-13 * max(1.0, np.abs(Ys).max())
        for flags in (hmx.HM_FAR_FROM_POINTS, both):
            Yp = run(hmx, M, W, flags)
            assert rel(Yp, Yref) <= 1e-10
            np.testing.assert_allclose(Yp, Yref, rtol=0, atol=1e-12 * max(1.0, np.abs(Yref).max()))
            np.testing.assert_allclose(Yp, Ys, rtol=0, atol=tol)


def test_far_from_points_tree_order_and_repeat(hmx):
    w, X, H = built("mix8")
    M = hmx.hm_load_compressed_mem(H, 0)
    hmx.hm_set_points(M, X, w.kernel, w.h)
    W = wl.gen_w(w, Q=64, seed=8)
    Yref = H.eval(W)
    f = hmx.HM_FAR_FROM_POINTS
    Y1, Y2 = run(hmx, M, W, f), run(hmx, M, W, f)
    np.testing.assert_array_equal(Y1, Y2)  # deterministic
    perm = H.perm
    Yt = run(hmx, M, np.ascontiguousarray(W[perm]), f | hmx.HM_TREE_ORDER)
    np.testing.assert_allclose(Yt, Yref[perm], rtol=0, atol=1e-12 * np.abs(Yref).max())


def test_far_from_points_needs_skeletons(hmx):
    w, X, H = built("c1")
    M = hmx.hm_load_compressed_mem(H, 0, skeletons=False)
    hmx.hm_set_points(M, X, w.kernel, w.h)
    W = wl.gen_w(w)
    with pytest.raises(hmx.HMError):  # the skeletons were not loaded
        run(hmx, M, W, hmx.HM_FAR_FROM_POINTS)
    Y = run(hmx, M, W, hmx.HM_NEAR_FROM_POINTS)  # the near field needs none
    assert rel(Y, H.eval(W)) <= 1e-10
    with pytest.raises(hmx.HMError):
        hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.HM_LOAD_NO_FAR_BLOCKS,
                                   skeletons=False)
    M2 = hmx.hm_load_compressed_mem(H, 0)
    with pytest.raises(hmx.HMError):  # no points set yet
        run(hmx, M2, W, hmx.HM_FAR_FROM_POINTS)


def test_load_without_near_or_far_blocks(hmx):
    w, X, H = built("mix8")
    full = hmx.hm_load_compressed_mem(H, 0)
    fp64 = hmx.precbit(hmx.HM_PREC_FP64)
    Mf = hmx.hm_load_compressed_mem(H, 0, fp64 | hmx.HM_LOAD_NO_FAR_BLOCKS)
    Mb = hmx.hm_load_compressed_mem(H, 0, fp64 | hmx.HM_LOAD_NO_FAR_BLOCKS | hmx.HM_LOAD_NO_NEAR_BLOCKS)
    st = H.stats()
    full_b = hmx.hm_info(full)["bytes_fp64"]
    assert full_b - hmx.hm_info(Mf)["bytes_fp64"] >= 8 * st["E_B"]
    assert full_b - hmx.hm_info(Mb)["bytes_fp64"] >= 8 * (st["E_B"] + st["E_D"])
    W = wl.gen_w(w, Q=48, seed=12)
    Yref = H.eval(W)
    Ys = run(hmx, full, W, 0)
    with pytest.raises(hmx.HMError):  # the stored far blocks are not there
        run(hmx, Mf, W, 0)
    with pytest.raises(hmx.HMError):
        run(hmx, Mb, W, hmx.HM_FAR_FROM_POINTS)  # nor the near blocks (and no points yet)
    for M, flags in ((Mf, hmx.HM_FAR_FROM_POINTS), (Mb, hmx.HM_FAR_FROM_POINTS | hmx.HM_NEAR_FROM_POINTS)):
        hmx.hm_set_points(M, X, w.kernel, w.h)
        Y = run(hmx, M, W, flags)
        assert rel(Y, Yref) <= 1e-10
        np.testing.assert_allclose(Y, Ys, rtol=0, atol=1e-13 * np.abs(Yref).max())
    with pytest.raises(hmx.HMError):  # FP64 store only
        hmx.hm_load_compressed_mem(H, 0, fp64 | hmx.HM_LOAD_NO_FAR_BLOCKS | hmx.precbit(hmx.HM_PREC_FP32))
    with pytest.raises(hmx.HMError):  # the batched form reads stored blocks
        hmx.hm_batch_create([Mf], [16])
