"""Matrix-free near field on the GPU: with HM_NEAR_FROM_POINTS the FP64
task-graph launch computes every near block K(X[I_a], X[I_b]) (Section 2.1)
from the points inside its product tiles instead of reading it from the
device store.  Checked against the CPU FP64 oracle's tree walk (which reads
the near blocks it computed at compression) to the FP64 bar, and against the
stored-block path on the same inputs; the only differences are the device's
exp/sqrt rounding and the summation order."""
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
    "single_node": wl.small("single_node", N=100, d=3, m=128, Q=5),
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
def test_near_from_points_matches_oracle(hmx, name):
    w, X, H = built(name)
    M = hmx.hm_load_compressed_mem(H, 0)
    hmx.hm_set_points(M, X, w.kernel, w.h)
    for Q in (w.Q, 40, 300):  # 40: the 64-column tile, run at 128 columns in this mode
        _say(f"[near-points] case={name} N={w.N} d={w.d} Q={Q}")
        W = wl.gen_w(w, Q=Q, seed=500 + Q)
        Yp = run(hmx, M, W, hmx.HM_NEAR_FROM_POINTS)
        Yref = H.eval(W)
        assert rel(Yp, Yref) <= 1e-10
        np.testing.assert_allclose(Yp, Yref, rtol=0, atol=1e-12 * max(1.0, np.abs(Yref).max()))
        Ys = run(hmx, M, W, 0)  # stored near blocks, same launch otherwise
        np.testing.assert_allclose(Yp, Ys, rtol=0, atol=1e-13 * max(1.0, np.abs(Ys).max()))


def test_near_from_points_tree_order_and_repeat(hmx):
    w, X, H = built("mix8")
    M = hmx.hm_load_compressed_mem(H, 0)
    hmx.hm_set_points(M, X, w.kernel, w.h)
    hmx.hm_set_points(M, X, w.kernel, w.h)  # replacing the points is allowed
    W = wl.gen_w(w, Q=64, seed=7)
    Yref = H.eval(W)
    Y1 = run(hmx, M, W, hmx.HM_NEAR_FROM_POINTS)
    Y2 = run(hmx, M, W, hmx.HM_NEAR_FROM_POINTS)
    np.testing.assert_array_equal(Y1, Y2)  # deterministic
    perm = H.perm
    Yt = run(hmx, M, np.ascontiguousarray(W[perm]), hmx.HM_NEAR_FROM_POINTS | hmx.HM_TREE_ORDER)
    np.testing.assert_allclose(Yt, Yref[perm], rtol=0, atol=1e-12 * np.abs(Yref).max())


def test_near_from_points_rejects_bad_use(hmx):
    w, X, H = built("c1")
    M = hmx.hm_load_compressed_mem(H, 0, hmx.precbit(hmx.HM_PREC_FP64) | hmx.precbit(hmx.HM_PREC_FP32))
    W = wl.gen_w(w)
    with pytest.raises(hmx.HMError):  # no points set
        run(hmx, M, W, hmx.HM_NEAR_FROM_POINTS)
    with pytest.raises(hmx.HMError):  # d above 64
        hmx.hm_set_points(M, np.zeros((w.N, 65)), w.kernel, w.h)
    with pytest.raises(hmx.HMError):  # unknown kernel
        hmx.hm_set_points(M, X, 7, w.h)
    with pytest.raises(hmx.HMError):  # h <= 0
        hmx.hm_set_points(M, X, w.kernel, 0.0)
    hmx.hm_set_points(M, X, w.kernel, w.h)
    W32 = torch.from_numpy(W).to("cuda", torch.float32)
    with pytest.raises(hmx.HMError):  # FP64 only
        hmx.hm_eval(M, W32, torch.empty_like(W32), flags=hmx.HM_NEAR_FROM_POINTS)


def test_load_without_near_blocks(hmx):
    w, X, H = built("mix8")
    full = hmx.hm_load_compressed_mem(H, 0)
    bits = hmx.precbit(hmx.HM_PREC_FP64) | hmx.HM_LOAD_NO_NEAR_BLOCKS
    M = hmx.hm_load_compressed_mem(H, 0, bits)
    # the near blocks' device memory is not allocated (each block is stored
    # padded, so at least 8 E_D bytes are saved)
    saved = hmx.hm_info(full)["bytes_fp64"] - hmx.hm_info(M)["bytes_fp64"]
    assert saved >= 8 * H.stats()["E_D"]
    W = wl.gen_w(w, Q=48, seed=11)
    with pytest.raises(hmx.HMError):  # the stored near blocks are not there
        run(hmx, M, W, 0)
    with pytest.raises(hmx.HMError):  # nor the points yet
        run(hmx, M, W, hmx.HM_NEAR_FROM_POINTS)
    hmx.hm_set_points(M, X, w.kernel, w.h)
    Y = run(hmx, M, W, hmx.HM_NEAR_FROM_POINTS)
    Yref = H.eval(W)
    assert rel(Y, Yref) <= 1e-10
    np.testing.assert_allclose(Y, run(hmx, full, W, 0), rtol=0, atol=1e-13 * np.abs(Yref).max())
    with pytest.raises(hmx.HMError):  # FP64 store only
        hmx.hm_load_compressed_mem(H, 0, bits | hmx.precbit(hmx.HM_PREC_FP32))
    with pytest.raises(hmx.HMError):  # the batched form reads stored blocks
        hmx.hm_batch_create([M], [16])
