"""hm_eval_noalloc (the evaluation whose per-call device memory lives in the
library's fixed device array) through the C ABI, against hm_eval on the same
matrix and W: bitwise equal (same kernels, tiles and summation order) and
within the FP64 parity bar of the oracle (<= 1e-10 relative, Frobenius).
Two calls in a row, the second on a smaller matrix and a narrower W, so that
the second runs over what the first left in the shared array; then FP32,
split BF16, the tree-order flag, blocks from points, and the refusals (no
task graph yet, too large for the array, unsupported flags)."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.helpers import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hmx():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1812_07152_amd as hmx
    return hmx


BIG = wl.small("na_big", N=4096, d=3, m=64, h=0.5, tol=1e-5, rmax=64, Q=40)
SMALL = wl.small("na_small", N=1500, d=8, points="mixture", m=40, h=1.0, Q=12)


def _case(w, hmx, prec_mask):
    X = wl.gen_points(w)
    H = OracleH2.from_workload(w, X)
    M = hmx.hm_load_compressed_mem(H, 0, prec_mask)
    return X, H, M


def _pair(hmx, M, W, **kw):
    """(hm_eval result, hm_eval_noalloc result) on the same W; the reference
    call also builds the task graph that the no-alloc call needs."""
    Wd = torch.from_numpy(W).cuda()
    Y0 = torch.full_like(Wd, float("nan"))
    Y1 = torch.full_like(Wd, float("nan"))
    hmx.hm_eval(M, Wd, Y0, **kw)
    hmx.hm_eval_noalloc(M, Wd, Y1, **kw)
    hmx.hm_check(M)
    return Y0.cpu().numpy(), Y1.cpu().numpy()


def test_noalloc_two_calls_fp64_then_smaller(hmx):
    f64 = hmx.precbit(hmx.HM_PREC_FP64)
    _say("[noalloc] fp64 N=4096 Q=40")
    _, Hb, Mb = _case(BIG, hmx, f64)
    Wb = wl.gen_w(BIG)
    ref, got = _pair(hmx, Mb, Wb)
    assert np.array_equal(ref, got)
    assert rel(got, Hb.eval(Wb)) <= 1e-10
    _say("[noalloc] fp64 N=1500 Q=12 after it")
    _, Hs, Ms = _case(SMALL, hmx, f64)
    Ws = wl.gen_w(SMALL)
    ref, got = _pair(hmx, Ms, Ws)
    assert np.array_equal(ref, got)
    assert rel(got, Hs.eval(Ws)) <= 1e-10
    # the big matrix again, narrower: the array still holds the last call's data
    _say("[noalloc] fp64 N=4096 Q=5 after it")
    W5 = wl.gen_w(BIG, Q=5, seed=9)
    ref, got = _pair(hmx, Mb, W5)
    assert np.array_equal(ref, got)
    assert rel(got, Hb.eval(W5)) <= 1e-10


def test_noalloc_fp32_mixed_and_tree_order(hmx):
    mask = hmx.precbit(hmx.HM_PREC_FP64) | hmx.precbit(hmx.HM_PREC_FP32) | hmx.precbit(hmx.HM_PREC_BF16X3)
    _, H, M = _case(BIG, hmx, mask)
    W = wl.gen_w(BIG)
    _say("[noalloc] split BF16 N=4096 Q=40")
    ref, got = _pair(hmx, M, W, prec=hmx.HM_PREC_BF16X3)
    assert np.array_equal(ref, got)
    assert rel(got, H.eval(W)) <= BIG.tol  # compressed at 1e-5: the split path meets the tol
    _say("[noalloc] fp32 N=4096 Q=40")
    W32 = W.astype(np.float32)
    ref, got = _pair(hmx, M, W32)
    assert np.array_equal(ref, got)
    assert rel(got.astype(np.float64), H.eval(W32.astype(np.float64))) <= 5e-6
    _say("[noalloc] fp64 tree order, then split BF16 on a narrower W")
    ref, got = _pair(hmx, M, W, flags=hmx.HM_TREE_ORDER)
    assert np.array_equal(ref, got)
    W7 = wl.gen_w(BIG, Q=7, seed=3)
    ref, got = _pair(hmx, M, W7, prec=hmx.HM_PREC_BF16X3)
    assert np.array_equal(ref, got)
    assert rel(got, H.eval(W7)) <= 5e-5


def test_noalloc_blocks_from_points(hmx):
    f64 = hmx.precbit(hmx.HM_PREC_FP64)
    X, H, M = _case(SMALL, hmx, f64 | hmx.HM_LOAD_NO_NEAR_BLOCKS | hmx.HM_LOAD_NO_FAR_BLOCKS)
    hmx.hm_set_points(M, X, SMALL.kernel, SMALL.h)
    W = wl.gen_w(SMALL)
    _say("[noalloc] near and far blocks from the points, N=1500 Q=12")
    ref, got = _pair(hmx, M, W, flags=hmx.HM_NEAR_FROM_POINTS | hmx.HM_FAR_FROM_POINTS)
    assert np.array_equal(ref, got)
    assert rel(got, H.eval(W)) <= 1e-10


def test_noalloc_refusals(hmx):
    f64 = hmx.precbit(hmx.HM_PREC_FP64)
    _, H, M = _case(SMALL, hmx, f64)
    W = torch.from_numpy(wl.gen_w(SMALL)).cuda()
    Y = torch.zeros_like(W)
    lib = hmx.hm.lib
    # no task graph for this width yet: refused, nothing written
    st = lib.hm_eval_noalloc(M, W.data_ptr(), W.stride(0), Y.data_ptr(), Y.stride(0), W.shape[1],
                             hmx.HM_F64, hmx.HM_PREC_FP64, 0, None)
    assert st == hmx.hm.HM_ERR_INVALID and "task graph" in hmx.hm_last_error()
    torch.cuda.synchronize()
    assert float(Y.abs().max()) == 0.0
    # more workspace than the fixed array: N * Q' * 8 > 64 MiB (refused before any lookup)
    Qbig = (hmx.HM_NOALLOC_SCRATCH_BYTES // (8 * SMALL.N)) + 256
    st = lib.hm_eval_noalloc(M, W.data_ptr(), Qbig, Y.data_ptr(), Qbig, Qbig, hmx.HM_F64, hmx.HM_PREC_FP64, 0, None)
    assert st == hmx.hm.HM_ERR_INVALID and "fixed" in hmx.hm_last_error()
    # launch-style and profiling flags are hm_eval's only
    hmx.hm_eval(M, W, Y)
    for fl in (hmx.HM_LEVEL_LAUNCHES, hmx.HM_PROFILE):
        st = lib.hm_eval_noalloc(M, W.data_ptr(), W.stride(0), Y.data_ptr(), Y.stride(0), W.shape[1],
                                 hmx.HM_F64, hmx.HM_PREC_FP64, fl, None)
        assert st == hmx.hm.HM_ERR_INVALID
    # Q = 0 is a no-op, as for hm_eval
    assert lib.hm_eval_noalloc(M, W.data_ptr(), 1, Y.data_ptr(), 1, 0, hmx.HM_F64, hmx.HM_PREC_FP64, 0,
                               None) == hmx.hm.HM_OK
    hmx.hm_check(M)
